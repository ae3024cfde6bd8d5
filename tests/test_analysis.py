"""Host post-processing (paper_2112_08479_amd.analysis) against the values the
paper prints and the properties that fix the scaling laws.

* Eq. 5-8 reproduce the four numbers printed in Sec. 3.1 (tests/golden).
* Each transition time is where the front velocities of the two phases meet
  (Eq. 2, 4 and Fr), and at Re_cr the slumping phase ends in both ways at once.
* Eq. 1 and 3 are the time integrals of Eq. 2 and 4.
* The Froude fit (Eq. 59) is exact on a straight line, ignores samples outside
  2.5 <= t~ <= 10 and agrees with the oracle's numpy.polyfit on noisy data.
* z+ (Eq. 60-61), the span average and the wall sums (Eq. 64, 66), Eq. 63.
"""
import os

import numpy as np
import pytest

from oracle import diag as odiag
from paper_2112_08479_amd import analysis as an

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "scaling_laws_sec3.txt")


def _printed():
    rows = {}
    with open(GOLDEN) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            q, fr, re_b, val, half = line.split()
            rows[q] = (float(fr), float(re_b), float(val), float(half))
    return rows


def test_transition_times_match_the_printed_values():
    r = _printed()
    fr, _, v, h = r["t_SI"]
    assert abs(an.t_slumping_inertial(fr) - v) <= h
    _, re_b, v, h = r["t_IV"]
    assert abs(an.t_inertial_viscous(re_b) - v) <= h
    fr, _, v, h = r["Re_cr"]
    assert abs(an.critical_reynolds(fr) - v) <= h
    fr, re_b, v, h = r["t_SV"]
    assert abs(an.t_slumping_viscous(fr, re_b) - v) <= h


@pytest.mark.parametrize("h0,x0", [(1.0, 1.0), (0.5, 2.0), (1.0, 0.25)])
@pytest.mark.parametrize("fr,re_b", [(0.37, 1000.0), (0.42, 5000.0), (0.44, 30000.0)])
def test_transitions_are_where_front_velocities_meet(fr, re_b, h0, x0):
    t_si = an.t_slumping_inertial(fr, h0, x0)
    t_sv = an.t_slumping_viscous(fr, re_b, h0, x0)
    t_iv = an.t_inertial_viscous(re_b, h0, x0)
    assert an.inertial_velocity(t_si, h0, x0) == pytest.approx(fr, rel=1e-12)
    assert an.viscous_velocity(t_sv, re_b, h0, x0) == pytest.approx(fr, rel=1e-12)
    assert an.inertial_velocity(t_iv, h0, x0) == pytest.approx(
        an.viscous_velocity(t_iv, re_b, h0, x0), rel=1e-12)
    re_cr = an.critical_reynolds(fr, h0, x0)
    assert an.t_slumping_viscous(fr, re_cr, h0, x0) == pytest.approx(t_si, rel=1e-12)
    phases, times = an.phase_sequence(fr, re_b, h0, x0)
    if re_b > re_cr:
        assert phases == ("slumping", "inertial", "viscous") and times[0] < times[1]
    else:
        assert phases == ("slumping", "viscous")


def test_phase_sequences_of_cases_2_and_4():
    # Sec. 3.1: Case 2 (Re_b 1000) goes straight from slumping to viscous,
    # Case 4 (Re_b 5000, above Re_cr = 3170) passes through an inertial phase
    assert an.phase_sequence(0.37, 1000.0)[0] == ("slumping", "viscous")
    assert an.phase_sequence(0.42, 5000.0)[0] == ("slumping", "inertial", "viscous")


def test_front_laws_integrate_the_velocity_laws():
    t, h = np.linspace(1.0, 40.0, 201), 1e-4
    for xf, uf in ((lambda s: an.inertial_front(s, 0.7, 1.3), an.inertial_velocity(t, 0.7, 1.3)),
                   (lambda s: an.viscous_front(s, 4000.0, 0.7, 1.3), an.viscous_velocity(t, 4000.0, 0.7, 1.3))):
        slope = (xf(t + h) - xf(t - h)) / (2 * h)        # central difference, error O(h^2)
        assert np.allclose(slope, uf, rtol=1e-7)


def test_froude_fit_is_exact_on_a_line_and_uses_only_its_window():
    t = np.linspace(0.0, 12.0, 241)
    x = 0.3 + 0.41 * t
    x_bent = np.where((t < 2.5) | (t > 10.0), x + 5.0 * np.sin(t), x)
    assert an.froude_number(t, x) == pytest.approx(0.41, rel=1e-13)
    assert an.froude_number(t, x_bent) == pytest.approx(0.41, rel=1e-13)
    with pytest.raises(ValueError):
        an.froude_number([0.0, 1.0], [0.0, 1.0])


def test_froude_fit_matches_the_oracle_fit_on_noisy_data():
    rng = np.random.default_rng(3)
    t = np.sort(rng.uniform(0.0, 12.0, 300))
    x = 0.37 * t + 0.02 * rng.standard_normal(t.size)
    assert an.froude_number(t, x) == pytest.approx(odiag.froude_number(t, x), rel=1e-12)


def test_hat_scaling_collapses_the_slumping_inertial_time():
    # Sec. 1: with t^ = t~ h0^(1/2) / x0 the transition time becomes
    # (2 xi_IP h0^(1/2) / (3 Fr))^3, whatever x0
    for h0, x0 in ((1.0, 1.0), (0.5, 3.0), (0.8, 0.6)):
        t_si = an.t_slumping_inertial(0.4, h0, x0)
        t_hat, _ = an.hat_scaling(t_si, 0.0, h0, x0)
        assert float(t_hat) == pytest.approx((2 * an.XI_IP * np.sqrt(h0) / (3 * 0.4)) ** 3, rel=1e-12)


def test_z_plus_wall_sums_and_l1_error():
    nu = 4e-4
    tau = np.array([[4 * nu * nu, -4 * nu * nu], [0.0, 16 * nu * nu]])
    # u_tau = 2 nu, 2 nu, 0, 4 nu at dz1 = 1/2 -> z+ = 1, 1, 0, 2
    assert np.allclose(an.z_plus(tau, nu), [[1.0, 1.0], [0.0, 2.0]], rtol=1e-14)
    rng = np.random.default_rng(0)
    f = rng.standard_normal((7, 33))
    assert np.allclose(an.span_average(f), f.sum(0) / 7, rtol=1e-14)
    assert an.span_friction_force(an.span_average(f)) * 7 == pytest.approx(an.friction_force(f), rel=1e-12)
    assert an.e_l1([2.0, -4.0], [1.0, -5.0]) == pytest.approx(0.375)
    assert np.allclose(an.rescaled_distance([1.0, 3.0], 1.0, 2.0), [0.0, 1.0])
