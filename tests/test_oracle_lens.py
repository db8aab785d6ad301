"""Pins of the oracle's Born lightcone projection."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import lens, pm
from oracle.cosmology import Cosmology, lens_prefactor


@pytest.fixture(scope="module")
def geom(cosmo):
    return lens.MapGeometry(32, 2.0, (1.0, 0.5), cosmo)


def test_single_particle_total_and_centroid(cosmo, geom):
    box, np_side = 1000.0, 10   # shell thinner than the box: one image
    a_far, a_near = 0.6, 0.7
    chi_far, chi_near = cosmo.chi(a_far), cosmo.chi(a_near)
    chi_p = 0.5 * (chi_far + chi_near)
    nz = math.floor(chi_p / box)
    th = np.array([0.2 * geom.dtheta * 7.3, -0.3 * geom.dtheta * 5.1])
    x = np.array([[0.5 * box + th[0] * chi_p], [0.5 * box + th[1] * chi_p],
                  [chi_p - nz * box]])
    out = lens.project_shell(x, a_far, a_near, cosmo, box, np_side, geom,
                             include_mean=False)
    a = cosmo.a_of_chi(chi_p)
    pref = lens_prefactor(cosmo.omega_m)
    for s, chis in enumerate(geom.chi_src):
        if chi_p >= chis:            # behind the source plane: no signal
            assert np.all(out[s] == 0.0)
            continue
        w = pref * (box / np_side) ** 3 * (chis - chi_p) / (
            chis * chi_p * a * geom.omega_pix)
        assert abs(out[s].sum() - w) < 1e-12 * w
        j = np.arange(geom.npix)
        t = th / geom.dtheta + 0.5 * geom.npix - 0.5
        c0 = np.sum(out[s].sum(axis=1) * j) / out[s].sum()
        c1 = np.sum(out[s].sum(axis=0) * j) / out[s].sum()
        assert abs(c0 - t[0]) < 1e-10 and abs(c1 - t[1]) < 1e-10


def test_beyond_source_gives_nothing(cosmo, geom):
    box = 200.0
    chi_s = geom.chi_src[1]  # z = 0.5
    a_far = cosmo.a_of_chi(chi_s + 150.0)
    a_near = cosmo.a_of_chi(chi_s + 10.0)
    x = W.random_positions(2000, box, seed=4)
    out = lens.project_shell(x, a_far, a_near, cosmo, box, 10, geom)
    assert np.all(out[1] == 0.0)
    assert np.any(out[0] != 0.0)


def test_shell_partition_of_static_field(cosmo, geom):
    """Every image in (chi(a_last), chi(a_first)] is counted exactly once."""
    box, np_side = 150.0, 12
    x = W.random_positions(np_side ** 3, box, seed=8)
    a = np.linspace(0.35, 1.0, 6)
    parts = sum(lens.project_shell(x, a[i], a[i + 1], cosmo, box, np_side, geom)
                for i in range(len(a) - 1))
    whole = lens.project_shell(x, a[0], a[-1], cosmo, box, np_side, geom)
    assert np.max(np.abs(parts - whole)) < 1e-12 * np.max(np.abs(whole))


def test_linear_in_particle_set(cosmo, geom):
    box = 150.0
    x = W.random_positions(3000, box, seed=10)
    f = lambda xx: lens.project_shell(xx, 0.5, 0.8, cosmo, box, 10, geom,
                                      include_mean=False)
    both = f(x)
    split = f(x[:, :1234]) + f(x[:, 1234:])
    assert np.max(np.abs(both - split)) < 1e-12 * np.max(np.abs(both))


def test_prefactor_scales_with_omega_m():
    assert lens_prefactor(0.3) == pytest.approx(5.0069e-8, rel=1e-4)
    assert lens_prefactor(0.6) == 2 * lens_prefactor(0.3)


def test_bilinear_adjoint_identity():
    rng = np.random.default_rng(2)
    t0 = rng.uniform(-2, 18, 500)
    t1 = rng.uniform(-2, 18, 500)
    w = rng.standard_normal(500)
    m = rng.standard_normal((16, 16))
    lhs = np.sum(lens.bilinear_paint(t0, t1, w, 16) * m)
    rhs = np.sum(w * lens.bilinear_gather(t0, t1, m))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_uniform_lattice_has_zero_mean_convergence(cosmo):
    """The unperturbed lattice projected through all shells gives mean kappa
    ~ 0: the particle term and the analytic mean term cancel.  The residual
    is the sampling error of the lattice inside the light cone (about 1e-3
    here); a dropped factor, a wrong a(chi) or chi power breaks it by O(1)."""
    np_side, box = 32, 128.0
    g = lens.MapGeometry(32, 6.0, (1.0,), cosmo)
    q = pm.lattice_positions(np_side, np_side, box)
    a = np.linspace(0.5, 1.0, 6)   # chi(0.5) is just beyond the source
    pos, mean = 0.0, 0.0
    for i in range(5):
        pos += lens.project_shell(q, a[i], a[i + 1], cosmo, box, np_side, g,
                                  include_mean=False).mean()
        mean += lens.shell_mean(cosmo, cosmo.chi(a[i + 1]), cosmo.chi(a[i]),
                                g.chi_src[0])
    assert pos > 0 and mean < 0
    assert abs(pos + mean) < 3e-3 * pos


def test_shell_mean_two_quadratures(cosmo):
    for lo, hi, cs in ((100.0, 400.0, 2312.68), (2000.0, 2600.0, 2312.68),
                       (5.0, 90.0, 1322.0)):
        m1 = lens.shell_mean(cosmo, lo, hi, cs)
        m2 = lens.shell_mean_adaptive(cosmo, lo, hi, cs)
        assert abs(m1 - m2) < 1e-11 * abs(m2)
