"""Local (per-node) collision operators (oracle; test infrastructure only).

All functions act on a batch of n nodes: flow populations f (Q, n) -- full
values, not deviations -- and scalar populations phi (P, n), float64.

Order of operations inside one node (collide-then-stream form of Eq. 17):
  1. moments: chi = sum phi (Eq. 27); rho = sum f (Eq. 19, compressible,
     rho = 1 + delta rho as in Eq. 52-53); j = sum c f; Boussinesq force
     F = g' chi e_g with e_g = (0,0,-1) (Eq. 11 in lattice units);
     u = (j + F/2) / rho (Eq. 20).
  2. Smagorinsky eddy viscosity from the pre-collision non-equilibrium stress
     (Eq. 32-34, read in the standard form nu_T = (C_s Delta)^2 |S|,
     |S| = sqrt(2 S:S), Delta = 1; tau_f solves the resulting quadratic
     exactly) and the scalar diffusivity D0 + nu_T / Sc_T (Eq. 35).
  3. flow collision: BGK with Guo forcing (Eq. 21-26) or cumulant (Eq. 54-58).
  4. scalar collision with the velocity of step 1: BGK (Eq. 28-29) on D3Q7 /
     D3Q6, or factorized central moments (Eq. 37-51) on D3Q27.
"""
import math

import torch

from . import ring


def _c(lat):
    return lat.c.T.contiguous()          # (3, Q)


def macroscopic(f, phi, P, extra_force=None):
    """Eq. 18-20, 27 and 11. Returns rho (n,), j (3,n), chi (n,), F (3,n), u (3,n)."""
    c = _c(P.flow)
    rho = f.sum(0)
    j = c @ f
    chi = phi.sum(0)
    F = torch.zeros_like(j)
    F[2] = -P.g_prime * chi
    bf = P.cfg.body_force
    for a in range(3):
        if bf[a] != 0.0:
            F[a] = F[a] + bf[a]
    u = (j + 0.5 * F) / rho
    return rho, j, chi, F, u


def smagorinsky_tau(pi_neq, rho, P, cs_smag):
    """Total relaxation time tau_f from the non-equilibrium stress (3,3,n).

    tau_f = (tau0 + sqrt(tau0^2 + 18 sqrt(2) C_s^2 sqrt(Q) / rho)) / 2,
    Q = Pi:Pi. This is the root of tau^2 - tau0 tau - 3 C_s^2 |S| tau = 0 with
    |S| tau = 3 sqrt(2 Q) / (2 rho) (strain from the stress, S = -Pi/(2 rho cs^2
    tau)), i.e. nu_T = (C_s)^2 |S| and tau_f = tau0 + 3 nu_T (Eq. 25, 32-34).
    The square root of Q uses a zero subgradient at Q = 0. With the
    configuration's smag_paper_form the closure is the one printed in Eq. 32,
    nu_T = C_s |S| (Delta = 1), so C_s enters where C_s^2 stands above.
    """
    if cs_smag == 0.0:
        return torch.full_like(rho, P.tau0)
    cs_term = cs_smag if P.cfg.smag_paper_form else cs_smag ** 2
    Q = (pi_neq * pi_neq).sum((0, 1))
    pos = Q > 0
    sq = torch.where(pos, torch.sqrt(torch.where(pos, Q, torch.ones_like(Q))),
                     torch.zeros_like(Q))
    return 0.5 * (P.tau0 + torch.sqrt(P.tau0 ** 2 + 18.0 * math.sqrt(2.0) * cs_term * sq / rho))


def scalar_tau(tau_f, P, sc_t):
    """tau_phi = 1/2 + (D0 + nu_T / Sc_T) / cs_phi^2 with nu_T = (tau_f - tau0) cs^2
    (Eq. 30, 35 read as adding the turbulent diffusivity to D0)."""
    nu_t = (tau_f - P.tau0) * P.flow.cs2
    return 0.5 + (P.d0 + nu_t / sc_t) / P.scal.cs2


def feq_q19(rho, u, lat):
    """Second-order equilibrium, Eq. 22 (any lattice with cs^2 = 1/3)."""
    cu = _c(lat).T @ u                   # (Q, n)
    uu = (u * u).sum(0)
    cs2 = lat.cs2
    return lat.w[:, None] * rho[None] * (1 + cu / cs2 + cu * cu / (2 * cs2 ** 2) - uu / (2 * cs2))


def guo_source(u, F, tau, lat):
    """Eq. 26: (1 - 1/(2 tau)) w [ (c - u)/cs^2 + (c.u) c / cs^4 ] . F"""
    c = _c(lat)
    cs2 = lat.cs2
    cF = c.T @ F
    cu = c.T @ u
    uF = (u * F).sum(0)
    return (1 - 0.5 / tau)[None] * lat.w[:, None] * ((cF - uF[None]) / cs2 + cu * cF / cs2 ** 2)


def collide_bgk(f, rho, u, F, P, cs_smag):
    """BGK + Guo (Eq. 21-26) with Smagorinsky tau (Eq. 32-34).
    Pi_neq = sum_q c c (f - f_eq) (Eq. 33, outer product)."""
    lat = P.flow
    feq = feq_q19(rho, u, lat)
    c = _c(lat)
    fneq = f - feq
    pi = torch.einsum('aq,bq,qn->abn', c, c, fneq)
    tau = smagorinsky_tau(pi, rho, P, cs_smag)
    fstar = f - (f - feq) / tau[None] + guo_source(u, F, tau, lat)
    return fstar, tau


def central_moments(f, u, lat):
    """kappa_abc = sum_q (c_x - u_x)^a (c_y - u_y)^b (c_z - u_z)^c f_q,
    a, b, c in {0,1,2} (Eq. 39 applied to f). Returns (3,3,3,n)."""
    kappa = torch.zeros(3, 3, 3, f.shape[1], dtype=f.dtype)
    for q, (cx, cy, cz) in enumerate(lat.c_list):
        dx, dy, dz = cx - u[0], cy - u[1], cz - u[2]
        px = torch.stack([torch.ones_like(dx), dx, dx * dx])
        py = torch.stack([torch.ones_like(dy), dy, dy * dy])
        pz = torch.stack([torch.ones_like(dz), dz, dz * dz])
        kappa = kappa + px[:, None, None] * py[None, :, None] * pz[None, None, :] * f[q]
    return kappa


def raw_moments(f, lat):
    """m_abc = sum_q c_x^a c_y^b c_z^c f_q, a, b, c in {0,1,2} (Eq. 18). (3,3,3,n)"""
    m = torch.zeros(3, 3, 3, f.shape[1], dtype=f.dtype)
    for q, c in enumerate(lat.c_list):
        for a in range(3):
            for b in range(3):
                for cc in range(3):
                    if (c[0] == 0 and a > 0) or (c[1] == 0 and b > 0) or (c[2] == 0 and cc > 0):
                        continue
                    m[a, b, cc] = m[a, b, cc] + (c[0] ** a) * (c[1] ** b) * (c[2] ** cc) * f[q]
    return m


def populations_from_raw(m, lat):
    """Inverse of raw_moments: f = M0^{-1} m, M0[abc, q] = c_x^a c_y^b c_z^c
    (nonsingular on D3Q27)."""
    c = lat.c
    M0 = torch.stack([c[:, 0] ** a * c[:, 1] ** b * c[:, 2] ** cc
                      for a in range(3) for b in range(3) for cc in range(3)])  # (27, Q)
    return torch.linalg.inv(M0) @ m.reshape(27, m.shape[-1])


def collide_cumulant(f, rho, j, F, P, cs_smag):
    """Cumulant collision on D3Q27 (Eq. 54-58).

    a. cumulants of f / rho from the logarithm of its moment generating
       function (Eq. 54), taken on the raw moments; the first-order cumulants
       are the mean velocity j / rho (Eq. 57) and every cumulant of order >= 2
       is independent of the frame;
    b. LES: Pi_neq = rho (C_ab - delta_ab / 3) from the second-order cumulants;
    c. relaxation C* = (1 - w) C + w C_eq (Eq. 55): the deviatoric second-order
       cumulants C_110, C_101, C_011, C_200 - C_020, C_200 - C_002 with
       w1 = 1/tau_f (Eq. 58) towards 0; the trace C_200 + C_020 + C_002 with
       omega_bulk towards 1 (= 3 cs^2); every cumulant of order 3..6 with
       omega3..omega6 towards 0, or, for the parametrised method the paper's
       VirtualFluids runs use, as in ``relax_parametrized``;
    d. density is conserved (Eq. 56) and the force enters the first-order
       cumulants: C*_1 = (j + F) / rho, so that sum c f* = j + F (Eq. 17);
    e. back through exp and the inverse of the moment map.
    """
    lat = P.flow
    cfg = P.cfg
    m = raw_moments(f, lat) / rho
    C = ring.cumulants_from_moments(m)
    idx2 = {(0, 0): (2, 0, 0), (1, 1): (0, 2, 0), (2, 2): (0, 0, 2),
            (0, 1): (1, 1, 0), (0, 2): (1, 0, 1), (1, 2): (0, 1, 1)}
    pi = torch.zeros(3, 3, f.shape[1], dtype=f.dtype)
    for (a, b), (i, jj, k) in idx2.items():
        v = rho * (C[i, jj, k] - (1.0 / 3.0 if a == b else 0.0))
        pi[a, b] = v
        pi[b, a] = v
    tau = smagorinsky_tau(pi, rho, P, cs_smag)
    w1 = 1.0 / tau
    w2 = cfg.omega_bulk
    Cs = C.clone()
    cxx, cyy, czz = C[2, 0, 0], C[0, 2, 0], C[0, 0, 2]
    dxy = (1 - w1) * (cxx - cyy)
    dxz = (1 - w1) * (cxx - czz)
    tr = (1 - w2) * (cxx + cyy + czz) + w2 * 1.0
    Cs[2, 0, 0] = (tr + dxy + dxz) / 3.0
    Cs[0, 2, 0] = (tr - 2.0 * dxy + dxz) / 3.0
    Cs[0, 0, 2] = (tr + dxy - 2.0 * dxz) / 3.0
    Cs[1, 1, 0] = (1 - w1) * C[1, 1, 0]
    Cs[1, 0, 1] = (1 - w1) * C[1, 0, 1]
    Cs[0, 1, 1] = (1 - w1) * C[0, 1, 1]
    if cfg.parametrized:
        relax_parametrized(C, Cs, w1, w2, cfg.limiter)
    else:
        rates = {3: cfg.omega3, 4: cfg.omega4, 5: cfg.omega5, 6: cfg.omega6}
        for i in range(3):
            for jj in range(3):
                for k in range(3):
                    o = i + jj + k
                    if o >= 3:
                        Cs[i, jj, k] = (1 - rates[o]) * C[i, jj, k]
    js = j + F
    Cs[1, 0, 0] = js[0] / rho
    Cs[0, 1, 0] = js[1] / rho
    Cs[0, 0, 1] = js[2] / rho
    fstar = populations_from_raw(ring.moments_from_cumulants(Cs) * rho, lat)
    return fstar, tau


def parametrized_rates(w1, w2):
    """Rates and coefficients of the parametrised cumulant method that the
    paper applies (Sec. 2.3, VirtualFluids; its reference 55: Geier, Pasquali
    and Schoenherr, J. Comput. Phys. 348, 2017). The third-order rates are
    chosen so that the leading error of the shear diffusion vanishes; A and B
    set the fourth-order equilibria. w1: shear rate (Eq. 58), w2: bulk rate.

    Returns (w_plus, w_minus, w_111, A, B): w_plus relaxes the sums
    C_120 + C_102, C_210 + C_012, C_201 + C_021; w_minus their differences;
    w_111 relaxes C_111. A and B are singular at w1 = w2.
    """
    w_plus = 8 * (w1 - 2) * (w2 * (3 * w1 - 1) - 5 * w1) / (
        8 * (5 - 2 * w1) * w1 + w2 * (8 + w1 * (9 * w1 - 26)))
    w_minus = 8 * (w1 - 2) * (w1 + w2 * (3 * w1 - 7)) / (
        w2 * (56 - 42 * w1 + 9 * w1 * w1) - 8 * w1)
    w_111 = 24 * (w1 - 2) * (4 * w1 * w1 + w1 * w2 * (18 - 13 * w1)
                             + w2 * w2 * (2 + w1 * (6 * w1 - 11))) / (
        16 * w1 * w1 * (w1 - 6) - 2 * w1 * w2 * (216 + 5 * w1 * (9 * w1 - 46))
        + w2 * w2 * (w1 * (3 * w1 - 10) * (15 * w1 - 28) - 48))
    den = (w1 - w2) * (w2 * (2 + 3 * w1) - 8 * w1)
    A = (4 * w1 * w1 + 2 * w1 * w2 * (w1 - 6) + w2 * w2 * (w1 * (10 - 3 * w1) - 4)) / den
    B = (4 * w1 * w2 * (9 * w1 - 16) - 4 * w1 * w1
         - 2 * w2 * w2 * (2 + 9 * w1 * (w1 - 2))) / (3 * den)
    return w_plus, w_minus, w_111, A, B


def velocity_gradients(C, w1, w2):
    """Velocity gradients estimated from the pre-collision second-order
    cumulants C (of f / rho) at first order of the Chapman-Enskog expansion:
    the non-equilibrium part of C_ab is -(d_a u_b + d_b u_a) / (3 w), with the
    shear rate w1 for the deviatoric part and the bulk rate w2 for the trace
    (whose equilibrium value is 3 cs^2 = 1). Returns
    (dxux, dyuy, dzuz, Dxy, Dxz, Dyz), D_ab = d_a u_b + d_b u_a."""
    cxx, cyy, czz = C[2, 0, 0], C[0, 2, 0], C[0, 0, 2]
    div = -1.5 * w2 * (cxx + cyy + czz - 1.0)           # d_a u_a
    dx_dy = -1.5 * w1 * (cxx - cyy)                     # d_x u_x - d_y u_y
    dx_dz = -1.5 * w1 * (cxx - czz)                     # d_x u_x - d_z u_z
    dxux = (div + dx_dy + dx_dz) / 3.0
    dyuy = dxux - dx_dy
    dzuz = dxux - dx_dz
    return (dxux, dyuy, dzuz, -3.0 * w1 * C[1, 1, 0], -3.0 * w1 * C[1, 0, 1],
            -3.0 * w1 * C[0, 1, 1])


def relax_parametrized(C, Cs, w1, w2, limiter):
    """Orders 3..6 of the parametrised cumulant collision (Eq. 55 with the
    rates and equilibria of ``parametrized_rates``), written into Cs.

    * third order: the sums and differences of the pairs (C_120, C_102),
      (C_210, C_012), (C_201, C_021) relax towards 0 with w_plus and w_minus,
      C_111 with w_111. With a limiter lambda > 0 each rate w becomes
      w + (1 - w) |X| / (|X| + lambda) for its own quantity X (cumulants of
      f / rho, so lambda plays the part of rho lambda for cumulants of f): large
      third-order cumulants relax at rate 1 (Sec. 2.3, the stabilised method);
    * fourth order relaxes with rate 1 onto equilibria proportional to the
      velocity gradients: C_220 = -(2/3)(1/w1 - 1/2) A (d_x u_x + d_y u_y),
      C_211 = -(1/3)(1/w1 - 1/2) B (d_y u_z + d_z u_y) and their permutations;
    * fifth and sixth order relax with rate 1 towards 0.
    """
    w_plus, w_minus, w_111, A, B = parametrized_rates(w1, w2)

    def keep(w, X):                      # 1 - (limited rate)
        if limiter > 0:
            a = X.abs()
            return (1 - w) * (1 - a / (a + limiter))
        return 1 - w

    for a, b in (((1, 2, 0), (1, 0, 2)), ((2, 1, 0), (0, 1, 2)), ((2, 0, 1), (0, 2, 1))):
        plus = C[a] + C[b]
        minus = C[a] - C[b]
        plus = keep(w_plus, plus) * plus
        minus = keep(w_minus, minus) * minus
        Cs[a] = 0.5 * (plus + minus)
        Cs[b] = 0.5 * (plus - minus)
    Cs[1, 1, 1] = keep(w_111, C[1, 1, 1]) * C[1, 1, 1]
    dxux, dyuy, dzuz, Dxy, Dxz, Dyz = velocity_gradients(C, w1, w2)
    h = 1.0 / w1 - 0.5
    Cs[2, 2, 0] = -(2.0 / 3.0) * h * A * (dxux + dyuy)
    Cs[2, 0, 2] = -(2.0 / 3.0) * h * A * (dxux + dzuz)
    Cs[0, 2, 2] = -(2.0 / 3.0) * h * A * (dyuy + dzuz)
    Cs[2, 1, 1] = -(1.0 / 3.0) * h * B * Dyz
    Cs[1, 2, 1] = -(1.0 / 3.0) * h * B * Dxz
    Cs[1, 1, 2] = -(1.0 / 3.0) * h * B * Dxy
    for idx in ((2, 2, 1), (2, 1, 2), (1, 2, 2), (2, 2, 2)):
        Cs[idx] = torch.zeros_like(C[idx])


def collide_scalar(phi, chi, u, tau_phi, P):
    """Eq. 28-29: phi* = phi - (phi - w chi (1 + c.u / cs_phi^2)) / tau_phi.
    Reading: cs_phi^2 is the scalar lattice's own sound speed squared (1/3 for
    D3Q6 as printed, 1/4 for D3Q7) so that sum c phi_eq = chi u."""
    lat = P.scal
    cu = _c(lat).T @ u
    peq = lat.w[:, None] * chi[None] * (1 + cu / lat.cs2)
    return phi - (phi - peq) / tau_phi[None]


# Factorized central moments (Eq. 40-49): M_abc = kappa_abc - k kappa_lower,
# where "lower" is the index with every 2 replaced by 0. The table lists the
# coefficient k per index pattern (any permutation of the axes); patterns
# without a 2 (Eq. 40-43) are the central moments themselves. Reading: Eq. 46
# prints 1/3 for the (220) pattern; 1/9 (the product of two equilibrium
# second moments 1/3, as in Eq. 47's 1/9 and Eq. 49's 1/27) is used.
FCM_SUBTRACT = {
    (2, 0, 0): 1.0 / 3.0,    # Eq. 44
    (2, 1, 0): 1.0 / 3.0,    # Eq. 45
    (2, 2, 0): 1.0 / 9.0,    # Eq. 46 (reading)
    (2, 2, 1): 1.0 / 9.0,    # Eq. 47
    (2, 1, 1): 1.0 / 3.0,    # Eq. 48
    (2, 2, 2): 1.0 / 27.0,   # Eq. 49
}


def _fcm_term(a, b, c):
    """(k, lower index) of Eq. 40-49 for index (a, b, c); k = 0 if none."""
    k = FCM_SUBTRACT.get(tuple(sorted((a, b, c), reverse=True)), 0.0)
    lower = tuple(0 if e == 2 else e for e in (a, b, c))
    return k, lower


def fcm_factorize(kappa):
    """Central moments kappa (3,3,3,n) -> factorized central moments M."""
    M = kappa.clone()
    for a in range(3):
        for b in range(3):
            for c in range(3):
                k, lo = _fcm_term(a, b, c)
                if k:
                    M[a, b, c] = kappa[a, b, c] - k * kappa[lo]
    return M


def fcm_unfactorize(M):
    """Inverse of fcm_factorize: kappa_abc = M_abc + k kappa_lower, lower
    indices first (they carry no 2, so kappa_lower = M_lower)."""
    kappa = M.clone()
    for a in range(3):
        for b in range(3):
            for c in range(3):
                k, lo = _fcm_term(a, b, c)
                if k:
                    kappa[a, b, c] = M[a, b, c] + k * M[lo]
    return kappa


def populations_from_central(kappa, u, lat):
    """Inverse of central_moments (Eq. 39) at every node: solve
    T(u) phi = kappa with T[abc, p] = prod_d (c_pd - u_d)^a_d."""
    n = kappa.shape[-1]
    c = lat.c.to(kappa.dtype)                                   # (Q, 3)
    d = c.T[:, :, None] - u[:, None, :]                         # (3, Q, n): c_pd - u_d
    pw = torch.stack([torch.ones_like(d), d, d * d])            # (3 powers, 3 axes, Q, n)
    T = torch.einsum('apn,bpn,cpn->nabcp', pw[:, 0], pw[:, 1], pw[:, 2]).reshape(n, 27, lat.Q)
    rhs = kappa.reshape(27, n).T.unsqueeze(-1)
    return torch.linalg.solve(T, rhs).squeeze(-1).T


def collide_fcm(phi, chi, u, tau_phi, P, omega_high=1.0):
    """Factorized-central-moment scalar collision on D3Q27 (Eq. 37-51).

    a. central moments of phi about the fluid velocity u (Eq. 38-39);
    b. factorized central moments (Eq. 40-49, table above);
    c. relaxation towards the zero equilibrium (Eq. 50): M_000 = chi is
       conserved; the first-order moments relax with omega_100 = 1/tau_phi,
       which gives D = (1/omega_100 - 1/2)/3 (Eq. 51); every other moment with
       omega_high. Reading: the paper gives no value for the other rates;
       1 (every non-conserved moment above first order reset to equilibrium)
       is the default;
    d. back through the inverse factorization and the inverse of Eq. 39.
    """
    lat = P.scal
    kappa = central_moments(phi, u, lat)
    M = fcm_factorize(kappa)
    w1 = 1.0 / tau_phi
    Ms = (1.0 - omega_high) * M
    Ms[0, 0, 0] = M[0, 0, 0]
    for idx in ((1, 0, 0), (0, 1, 0), (0, 0, 1)):
        Ms[idx] = (1.0 - w1) * M[idx]
    return populations_from_central(fcm_unfactorize(Ms), u, lat)


def collide(f, phi, P, cs_smag=None, sc_t=None):
    """One full local collision. cs_smag / sc_t may be tensors (for autograd)
    or None to take them from the configuration. Returns (f*, phi*)."""
    cfg = P.cfg
    cs = cfg.cs_smag if cs_smag is None else cs_smag
    sct = cfg.sc_t if sc_t is None else sc_t
    rho, j, chi, F, u = macroscopic(f, phi, P)
    if cfg.model in (0, 2):
        fstar, tau = collide_cumulant(f, rho, j, F, P, cs)
    else:
        fstar, tau = collide_bgk(f, rho, u, F, P, cs)
    tau_phi = scalar_tau(tau, P, sct)
    if cfg.model == 2:
        phistar = collide_fcm(phi, chi, u, tau_phi, P)
    else:
        phistar = collide_scalar(phi, chi, u, tau_phi, P)
    return fstar, phistar
