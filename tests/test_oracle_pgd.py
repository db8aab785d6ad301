"""Pins of the oracle's PGD correction (the package-design section's first
technique; its operator as read from the paper's PGD reference):
S = alpha R(x, IFFT(O_l O_s i k delta_hat / k^2)), O_l = exp(-k_l^2/k^2),
O_s = exp(-(k/k_s)^4), applied to the projected positions of every step."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import lens, pm
from oracle.cosmology import Cosmology


def _one_mode_lattice(np_side, box, m, amp):
    """Lattice displaced along axis 0 by amp sin(2 pi m q0 / L): its CIC
    density holds the modes +-m along axis 0 only (to first order in amp)."""
    q = pm.lattice_positions(np_side, np_side, box)
    x = q.copy()
    x[0] = np.mod(q[0] + amp * np.sin(2.0 * np.pi * m * q[0] / box), box)
    return x


@pytest.mark.parametrize("m", [1, 3])
def test_one_mode_displacement_is_the_filtered_force(m):
    """For one Fourier mode the PGD displacement is alpha O_l(k) O_s(k)
    times the PM force, k = 2 pi m / L: pins where the filter acts and the
    units of k."""
    np_side, box = 16, 100.0
    k_l, k_s, alpha = 0.08, 0.35, 1.7
    x = _one_mode_lattice(np_side, box, m, 1e-4)
    f = pm.particle_force(x, np_side, np_side, box)
    s = pm.pgd_displacement(x, np_side, np_side, box, alpha, k_l, k_s)
    k = 2.0 * np.pi * m / box
    expect = alpha * math.exp(-(k_l / k) ** 2) * math.exp(-(k / k_s) ** 4)
    big = np.abs(f[0]) > 0.5 * np.abs(f[0]).max()
    ratio = s[0, big] / f[0, big]
    assert np.max(np.abs(ratio / expect - 1.0)) < 1e-5
    # transverse components carry no signal
    assert np.abs(s[1:]).max() < 1e-9 * np.abs(s[0]).max()


def test_unit_filters_give_the_pm_force():
    np_side, nm, box = 8, 16, 40.0
    x = W.clustered_positions(np_side, nm, box, seed=61)
    f = pm.particle_force(x, np_side, nm, box)
    s = pm.pgd_displacement(x, np_side, nm, box, 0.3, 0.0, 1e30)
    assert np.max(np.abs(s - 0.3 * f)) < 1e-12 * np.abs(f).max()


def test_displacement_is_linear_in_alpha():
    np_side, nm, box = 8, 16, 40.0
    x = W.clustered_positions(np_side, nm, box, seed=62)
    s1 = pm.pgd_displacement(x, np_side, nm, box, 1.0, 0.1, 0.8)
    s2 = pm.pgd_displacement(x, np_side, nm, box, -2.5, 0.1, 0.8)
    assert np.max(np.abs(s2 + 2.5 * s1)) < 1e-12 * np.abs(s1).max()


def test_zero_amplitude_is_the_plain_run(cosmo):
    c = Cosmology(0.3)
    g = lens.MapGeometry(24, 3.0, (1.0,), c)
    noise = W.white_noise(8, 11)
    a_grid = np.linspace(0.3, 1.0, 3)
    k0, _, _ = lens.run_lensing(noise, c, 40.0, 8, a_grid, g)
    k1, _, _ = lens.run_lensing(noise, c, 40.0, 8, a_grid, g, pgd=(0.0, 1.0, 0.1, 1.0))
    np.testing.assert_array_equal(k1, k0)
    k2, _, _ = lens.run_lensing(noise, c, 40.0, 8, a_grid, g, pgd=(5.0, 1.0, 0.1, 1.0))
    assert np.abs(k2 - k0).max() > 1e-6 * np.abs(k0).max()
