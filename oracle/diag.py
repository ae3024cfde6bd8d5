"""Diagnostics of a pre-collision state (oracle; test infrastructure only).

mass M = sum rho; scalar mass X = sum chi.

Bottom-wall shear stress (Eq. 62): tau_w = mu du/dz at the wall, with a
second-order one-sided difference through the two nearest fluid nodes
(Sec. 3.2). With the half-way wall the nodes sit at distances 1/2 and 3/2 from
the wall where u = 0; the quadratic through (0, 0), (1/2, u0), (3/2, u1) has
slope (9 u0 - u1) / 3 at the wall. mu = rho_bar nu0 with rho_bar = 1
(Eq. 52). u is the streamwise component u_x (signed). Friction force F_w =
sum over the bottom layer of tau_w (Eq. 64, Delta x = 1);
F_w~ = F_w / (U_b^2 H^2).

Front (Sec. 3.1): span average chi_bar(i, k) = mean_j chi; column maximum
m(i) = max_k chi_bar(i, k); i* = the largest i with m(i) >= 0.02 (reading of
the right-to-left search for the first node above the threshold);
x_front = i* + 1/2 + (m(i*) - 0.02) / (m(i*) - m(i* + 1)) (linear
interpolation between node centres), N1 if i* = N1 - 1, 0 if no column
reaches the threshold. x_f = x_front - x0, x0 = gate index; x_f~ = x_f / N3.
"""
import torch

from . import lbm

THRESH = 0.02


def front_position(chi):
    """chi (N3, N2, N1) -> (x_front, i_star). Differentiable through chi."""
    nz, ny, nx = chi.shape
    chibar = chi.mean(1)                     # (N3, N1)
    m, _ = chibar.max(0)                     # (N1,)
    above = (m >= THRESH).nonzero()
    if above.numel() == 0:
        return chi.sum() * 0.0, -1
    i_star = int(above.max())
    if i_star == nx - 1:
        return chi.sum() * 0.0 + float(nx), i_star
    x = i_star + 0.5 + (m[i_star] - THRESH) / (m[i_star] - m[i_star + 1])
    return x, i_star


def wall_shear(u, P):
    """tau_w(j, i) = nu0 (9 u_x(i, j, z=0) - u_x(i, j, z=1)) / 3, shape (N2, N1),
    and its span average (N1,) (Sec. 3.2, the integrand of Eq. 66)."""
    tau = P.nu0 * (9.0 * u[0, 0] - u[0, 1]) / 3.0
    return tau, tau.mean(0)


def froude_number(t_nd, x_f_nd, t_lo=2.5, t_hi=10.0):
    """Eq. 59: the front velocity d x_f~ / d t~ over 2.5 <= t~ <= 10, taken as
    the least-squares slope of a straight line through the samples in that
    window (numpy.polyfit, degree 1)."""
    import numpy as np
    t = np.asarray(t_nd, dtype=np.float64)
    x = np.asarray(x_f_nd, dtype=np.float64)
    sel = (t >= t_lo) & (t <= t_hi)
    return float(np.polyfit(t[sel], x[sel], 1)[0])


def wall_friction(u, P):
    """F_w = sum_{i,j} nu0 (9 u_x(z=0) - u_x(z=1)) / 3 (u: (3, N3, N2, N1))."""
    return (P.nu0 * (9.0 * u[0, 0] - u[0, 1]) / 3.0).sum()


def diagnostics(f, phi, P, step=0, lock_fraction=0.125):
    rho, u, chi = lbm.moments(f, phi, P)
    x_front, _ = front_position(chi)
    nx = P.cfg.nx
    x0 = lbm.gate_index(nx, lock_fraction)
    umag = torch.sqrt((u * u).sum(0))
    fin = torch.isfinite(rho) & torch.isfinite(chi) & torch.isfinite(u).all(0)
    fw = float(wall_friction(u, P)) if P.cfg.nz >= 2 else 0.0
    x_front = float(x_front)
    return {
        'step': step,
        't_nd': step * P.u_b / P.H,
        'mass': float(rho.sum()),
        'chi_mass': float(chi.sum()),
        'fw': fw,
        'fw_nd': fw / (P.u_b ** 2 * P.H ** 2) if P.u_b > 0 else 0.0,
        'x_front': x_front,
        'x_f': x_front - x0,
        'x_f_nd': (x_front - x0) / P.H,
        'umax': float(umag.max()),
        'nonfinite': int((~fin).sum()),
    }
