"""Host-side post-processing of the lock-exchange diagnostics (numpy).

Every quantity here is computed from outputs of the library (the front series
x_f~(t~) of ``Lattice.diagnostics``, the wall shear stress of
``Lattice.wall_shear``); nothing here touches the populations.

Non-dimensional quantities carry a tilde in the paper: lengths in units of the
channel depth H, velocities in units of the buoyancy velocity
U_b = sqrt(g' H), times in units of H / U_b. h0~ and x0~ are the lock depth
and length (both 1 for the full-depth lock of length H).

Scaling laws (Sec. 1): slumping phase x_f~ = Fr t~; inertial phase Eq. 1-2
with the constant xi_IP; viscous phase Eq. 3-4 with xi_VP. The transition
times Eq. 5-7 are where the front velocities of two phases coincide, and the
critical Reynolds number Eq. 8 is where t_SI = t_SV. Defaults are the fitted
constants quoted in Sec. 1: xi_IP = 1.47, xi_VP = 3.2.
"""
import numpy as np

XI_IP = 1.47
XI_VP = 3.2


def froude_number(t_nd, x_f_nd, t_lo=2.5, t_hi=10.0):
    """Eq. 59: the constant front velocity of the slumping phase, the slope of
    the ordinary least-squares line x_f~ = a + Fr t~ through the samples with
    t_lo <= t~ <= t_hi (closed form: cov(t, x) / var(t))."""
    t = np.asarray(t_nd, dtype=np.float64)
    x = np.asarray(x_f_nd, dtype=np.float64)
    sel = (t >= t_lo) & (t <= t_hi)
    if sel.sum() < 2:
        raise ValueError("fewer than two samples in the fitting window")
    t, x = t[sel], x[sel]
    dt = t - t.mean()
    return float((dt * (x - x.mean())).sum() / (dt * dt).sum())


def front_velocity(t_nd, x_f_nd):
    """u_f~ = d x_f~ / d t~ by central differences of the sampled series
    (one-sided at the ends)."""
    return np.gradient(np.asarray(x_f_nd, dtype=np.float64), np.asarray(t_nd, dtype=np.float64))


def inertial_front(t, h0=1.0, x0=1.0, xi_ip=XI_IP):
    """Eq. 1: x_f~ = xi_IP (h0~ x0~)^(1/3) t~^(2/3)."""
    return xi_ip * (h0 * x0) ** (1.0 / 3.0) * np.asarray(t, dtype=np.float64) ** (2.0 / 3.0)


def inertial_velocity(t, h0=1.0, x0=1.0, xi_ip=XI_IP):
    """Eq. 2: u_f~ = (2/3) xi_IP (h0~ x0~)^(1/3) t~^(-1/3)."""
    return 2.0 / 3.0 * xi_ip * (h0 * x0) ** (1.0 / 3.0) * np.asarray(t, dtype=np.float64) ** (-1.0 / 3.0)


def viscous_front(t, re_b, h0=1.0, x0=1.0, xi_vp=XI_VP):
    """Eq. 3: x_f~ = xi_VP (h0~^3 x0~^3 Re_b)^(1/5) t~^(1/5)."""
    return xi_vp * (h0 ** 3 * x0 ** 3 * re_b) ** 0.2 * np.asarray(t, dtype=np.float64) ** 0.2


def viscous_velocity(t, re_b, h0=1.0, x0=1.0, xi_vp=XI_VP):
    """Eq. 4: u_f~ = (1/5) xi_VP (h0~^3 x0~^3 Re_b)^(1/5) t~^(-4/5)."""
    return 0.2 * xi_vp * (h0 ** 3 * x0 ** 3 * re_b) ** 0.2 * np.asarray(t, dtype=np.float64) ** (-0.8)


def t_slumping_inertial(fr, h0=1.0, x0=1.0, xi_ip=XI_IP):
    """Eq. 5: t_SI~ = (2 xi_IP / (3 Fr))^3 h0~ x0~."""
    return (2.0 * xi_ip / (3.0 * fr)) ** 3 * h0 * x0


def t_slumping_viscous(fr, re_b, h0=1.0, x0=1.0, xi_vp=XI_VP):
    """Eq. 6: t_SV~ = (xi_VP / 5)^(5/4) (h0~ x0~)^(3/4) Fr^(-5/4) Re_b^(1/4)."""
    return (xi_vp / 5.0) ** 1.25 * (h0 * x0) ** 0.75 / fr ** 1.25 * re_b ** 0.25


def t_inertial_viscous(re_b, h0=1.0, x0=1.0, xi_ip=XI_IP, xi_vp=XI_VP):
    """Eq. 7: t_IV~ = (3 xi_VP / (10 xi_IP))^(15/7) (h0~ x0~)^(4/7) Re_b^(3/7)."""
    return (3.0 * xi_vp / (10.0 * xi_ip)) ** (15.0 / 7.0) * (h0 * x0) ** (4.0 / 7.0) * re_b ** (3.0 / 7.0)


def critical_reynolds(fr, h0=1.0, x0=1.0, xi_ip=XI_IP, xi_vp=XI_VP):
    """Eq. 8: Re_cr = (2 xi_IP / (3 Fr))^12 (5 Fr / xi_VP)^5 h0~ x0~; above it
    the current passes through an inertial phase (t_SI < t_SV)."""
    return (2.0 * xi_ip / (3.0 * fr)) ** 12 * (5.0 * fr / xi_vp) ** 5 * h0 * x0


def phase_sequence(fr, re_b, h0=1.0, x0=1.0, xi_ip=XI_IP, xi_vp=XI_VP):
    """The phases the scaling laws predict and their transition times:
    ('slumping', 'inertial', 'viscous') with (t_SI, t_IV) when t_SI < t_SV,
    else ('slumping', 'viscous') with (t_SV,)."""
    t_si = t_slumping_inertial(fr, h0, x0, xi_ip)
    t_sv = t_slumping_viscous(fr, re_b, h0, x0, xi_vp)
    if t_si < t_sv:
        return ("slumping", "inertial", "viscous"), (t_si, t_inertial_viscous(re_b, h0, x0, xi_ip, xi_vp))
    return ("slumping", "viscous"), (t_sv,)


def hat_scaling(t_nd, u_nd, h0=1.0, x0=1.0):
    """Rescaling of Sec. 1 by the lock: u^ = u~ / h0~^(1/2),
    t^ = t~ h0~^(1/2) / x0~."""
    return (np.asarray(t_nd, dtype=np.float64) * np.sqrt(h0) / x0,
            np.asarray(u_nd, dtype=np.float64) / np.sqrt(h0))


def shear_nd(tau_lu, u_b):
    """tau_w~ = tau_w / (rho_bar U_b^2) with rho_bar = 1 (lattice units in)."""
    return np.asarray(tau_lu, dtype=np.float64) / (u_b * u_b)


def z_plus(tau_lu, nu, dz1=0.5, rho=1.0):
    """Eq. 60-61 in lattice units: u_tau = sqrt(|tau_w| / rho),
    z+ = u_tau dz1 / nu; dz1 = 1/2 is the distance from the half-way wall to
    the wall-adjacent node. Both sides of Eq. 60 are ratios, so lattice and
    non-dimensional units give the same z+."""
    return np.sqrt(np.abs(np.asarray(tau_lu, dtype=np.float64)) / rho) * dz1 / nu


def span_average(tau_xy):
    """tau_bar(x) = (1/L2) int tau_w dy: the mean over the span axis of a
    (ny, nx) field."""
    return np.asarray(tau_xy, dtype=np.float64).mean(axis=0)


def friction_force(tau_xy, dx=1.0):
    """Eq. 64: F_w = sum over the wall of tau_w dx dy for a (ny, nx) field."""
    return float(np.asarray(tau_xy, dtype=np.float64).sum() * dx * dx)


def span_friction_force(tau_bar, dx=1.0):
    """Eq. 66: F_w bar = int tau_bar dx for the span-averaged profile."""
    return float(np.asarray(tau_bar, dtype=np.float64).sum() * dx)


def rescaled_distance(x_nd, x0_nd, x_f_nd):
    """Streamwise coordinate of the tau_bar plots of Sec. 3.2,
    (x~ - x0~) / x_f~: the front sits at 1."""
    return (np.asarray(x_nd, dtype=np.float64) - x0_nd) / x_f_nd


def e_l1(reference, model):
    """Eq. 63 / 65: mean over the sample times of |(ref - model) / ref|."""
    r = np.asarray(reference, dtype=np.float64)
    m = np.asarray(model, dtype=np.float64)
    return float(np.mean(np.abs((r - m) / r)))
