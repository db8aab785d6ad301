"""Pins of the oracle's background, growth, time factors and P(k).

Each test checks the oracle against something other than itself: a
closed form (Einstein-de Sitter), a second independent quadrature, the
growth ODE, an asymptotic limit, or an exact symmetry.
"""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle.cosmology import C_OVER_H0, Cosmology


def test_eds_distance_closed_form():
    c = Cosmology(1.0)
    for a in (0.01, 0.1, 0.25, 0.5, 0.9):
        exact = 2.0 * C_OVER_H0 * (1.0 - math.sqrt(a))
        assert abs(c.chi(a) - exact) <= 1e-11 * exact
        assert abs(c.chi_vec(a) - exact) <= 1e-11 * exact
        z = 1.0 / a - 1.0
        assert abs(c.chi_of_z(z) - exact) <= 1e-11 * exact


def test_eds_growth_and_factors_closed_form():
    c = Cosmology(1.0)
    for a in (0.02, 0.3, 0.77):
        assert abs(c.D(a) - a) <= 1e-12
        assert abs(c.gp(a) - a ** 1.5) <= 1e-12
    a_s, a_e, a_r = 0.3, 0.4, 0.35
    assert abs(c.drift_factor(a_s, a_e, a_r) - (a_e - a_s) / a_r ** 1.5) < 1e-12
    assert abs(c.kick_factor(a_s, a_e, a_r)
               - (a_e ** 1.5 - a_s ** 1.5) / a_r) < 1e-12


@pytest.mark.parametrize("om", [0.25, 0.3, 0.35])
def test_three_distance_quadratures_agree(om):
    c = Cosmology(om)
    for a in (0.01, 0.1, 0.5, 0.95):
        d1 = c.chi(a)                     # adaptive, over a
        d2 = float(c.chi_vec(a))          # Gauss-Legendre, substituted
        d3 = c.chi_of_z(1.0 / a - 1.0)    # adaptive, over z (paper's form)
        assert abs(d1 - d2) <= 1e-12 * d1
        assert abs(d1 - d3) <= 1e-12 * d1


def test_a_of_chi_inverts(cosmo):
    chis = np.array([0.5, 50.0, 571.71, 2312.68, 8000.0])
    a_brent = np.array([cosmo.a_of_chi(v) for v in chis])
    a_newton = cosmo.a_of_chi_vec(chis)
    assert np.max(np.abs(a_brent - a_newton)) < 1e-12
    back = np.array([cosmo.chi(a) for a in a_brent])
    assert np.max(np.abs(back - chis) / chis) < 1e-11


@pytest.mark.parametrize("om", [0.25, 0.3, 0.35])
def test_growth_ode_residual(om):
    """d g_p / da = (3/2) Om D / (a^2 E): the linear growth equation."""
    c = Cosmology(om)
    for a in (0.02, 0.2, 0.6, 1.0):
        h = 1e-4 * a
        lhs = (c.gp(a + h) - c.gp(a - h)) / (2 * h)
        rhs = 1.5 * om * c.D(a) / (a * a * float(c.E(a)))
        assert abs(lhs - rhs) <= 1e-7 * abs(rhs)


def test_growth_linear_at_early_times(cosmo):
    r1 = cosmo.D(1e-3) / 1e-3
    r2 = cosmo.D(2e-3) / 2e-3
    assert abs(r1 - r2) < 1e-7 * r1
    # the growth rate approximation f = Om(a)^0.55 holds to about 1%
    a = 0.5
    h = 1e-5
    f = (math.log(cosmo.D(a + h)) - math.log(cosmo.D(a - h))) / (
        math.log(a + h) - math.log(a - h))
    om_a = cosmo.omega_m / a ** 3 / float(cosmo.E(a)) ** 2
    assert abs(f / om_a ** 0.55 - 1.0) < 0.01


def test_time_factors_antisymmetric_and_leapfrog_limit(cosmo):
    a_s, a_e, a_r = 0.31, 0.37, 0.34
    assert cosmo.kick_factor(a_s, a_e, a_r) == -cosmo.kick_factor(a_e, a_s, a_r)
    assert cosmo.drift_factor(a_s, a_e, a_r) == -cosmo.drift_factor(a_e, a_s, a_r)
    # small steps: K -> (3/2) Om int da/(a^2 E), Dr -> int da/(a^3 E)
    for da in (1e-2, 5e-3):
        a0 = 0.5
        a1 = a0 + da
        am = 0.5 * (a0 + a1)
        k_std = 1.5 * cosmo.omega_m * integrate.quad(
            lambda a: 1.0 / (a * a * float(cosmo.E(a))), a0, a1, epsrel=1e-13)[0]
        d_std = integrate.quad(
            lambda a: 1.0 / (a ** 3 * float(cosmo.E(a))), a0, a1, epsrel=1e-13)[0]
        assert abs(cosmo.kick_factor(a0, a1, am) / k_std - 1) < 2 * da * da
        assert abs(cosmo.drift_factor(a0, a1, am) / d_std - 1) < 2 * da * da


def test_transfer_limits(cosmo):
    assert abs(float(cosmo.transfer_nowiggle(1e-6)) - 1.0) < 1e-5
    k = np.array([1e-5, 2e-5])
    p = cosmo.pk_linear(k)
    assert abs(math.log(p[1] / p[0]) / math.log(2.0) - cosmo.n_s) < 1e-3
    t = cosmo.transfer_nowiggle(np.logspace(-4, 2, 50))
    assert np.all(np.diff(t) < 0)  # monotone suppression


def test_sigma8_normalisation_independent_quadrature(cosmo):
    """Recompute sigma8 with a plain trapezoid on a fine log grid."""
    lnk = np.linspace(math.log(1e-6), math.log(300.0), 400001)
    k = np.exp(lnk)
    w = cosmo.tophat_window(8.0 * k)
    integrand = k ** 3 * cosmo.pk_linear(k) * w * w / (2 * math.pi ** 2)
    s8 = math.sqrt(np.trapezoid(integrand, lnk))
    assert abs(s8 - cosmo.sigma8) < 1e-6


def test_source_plane_distances(cosmo):
    """chi(z) at the source planes of the workloads (independent check of
    the order of magnitude, from the quadrature over z)."""
    chis = [cosmo.chi_of_z(z) for z in (0.5, 1.0, 1.5, 2.0)]
    assert np.allclose(chis, [1322.04, 2312.68, 3054.70, 3625.90], atol=0.01)
