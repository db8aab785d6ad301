"""Pins of the oracle's hand-derived reverse pass: central finite differences
of the forward oracle and dot-product identities."""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint, lens, pm
from oracle.cosmology import Cosmology


@pytest.fixture(scope="module")
def small():
    c = Cosmology(0.3)
    return c, 8, 16, 40.0


def test_force_operator_transpose_dot_product():
    rng = np.random.default_rng(3)
    n, box = 12, 30.0
    rho = 1.0 + rng.standard_normal((n, n, n))
    mbar = rng.standard_normal((3, n, n, n))
    lhs = np.sum(pm.force_mesh(rho, box) * mbar)
    rhs = np.sum((rho - 1.0) * adjoint.force_operator_transpose(mbar, box))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_cic_gradient_matches_finite_difference():
    rng = np.random.default_rng(4)
    n, box = 10, 20.0
    mesh = rng.standard_normal((n, n, n))
    x = W.random_positions(50, box, seed=5)
    g = adjoint.cic_gradient_gather(x, mesh, box)
    eps = 1e-7
    for d in range(3):
        dx = np.zeros_like(x)
        dx[d] = eps
        fd = (pm.cic_readout(x + dx, mesh, box) - pm.cic_readout(x - dx, mesh, box)) / (2 * eps)
        assert np.max(np.abs(fd - g[d])) < 1e-6 * np.max(np.abs(g))


def test_force_vjp_matches_finite_difference(small):
    _, np_side, nm, box = small
    x = W.clustered_positions(np_side, nm, box, seed=6)
    rng = np.random.default_rng(7)
    fbar = rng.standard_normal(x.shape)
    v = rng.standard_normal(x.shape)
    eps = 1e-7
    fp = pm.particle_force(np.mod(x + eps * v, box), np_side, nm, box)
    fm = pm.particle_force(np.mod(x - eps * v, box), np_side, nm, box)
    fd = np.sum(fbar * (fp - fm)) / (2 * eps)
    ad = np.sum(adjoint.force_vjp(x, fbar, np_side, nm, box) * v)
    assert abs(fd - ad) < 1e-6 * abs(ad)


def test_lens_vjp_matches_finite_difference():
    c = Cosmology(0.3)
    box, np_side = 64.0, 12
    geom = lens.MapGeometry(24, 4.0, (1.0, 2.0), c)
    x = W.clustered_positions(np_side, 24, box, seed=8)
    rng = np.random.default_rng(9)
    kbar = rng.standard_normal((2, 24, 24))
    v = rng.standard_normal(x.shape)
    a_far, a_near = 0.55, 0.7
    eps = 1e-7
    f = lambda xx: np.sum(kbar * lens.project_shell(xx, a_far, a_near, c, box, np_side, geom,
                                                    include_mean=False))
    fd = (f(np.mod(x + eps * v, box)) - f(np.mod(x - eps * v, box))) / (2 * eps)
    ad = np.sum(adjoint.lens_vjp(x, a_far, a_near, kbar, c, box, np_side, geom) * v)
    assert abs(fd - ad) < 1e-6 * abs(ad)


def test_ic_transpose_dot_product():
    c = Cosmology(0.3)
    np_side, box = 12, 50.0
    rng = np.random.default_rng(10)
    w = rng.standard_normal((np_side,) * 3)
    sbar = rng.standard_normal((3, np_side ** 3))
    lhs = np.sum(pm.zeldovich_displacement(w, c, box) * sbar)
    rhs = np.sum(w * adjoint.ic_displacement_transpose(sbar, c, box))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def _loss_setup():
    c = Cosmology(0.3)
    np_side, nm, box = 8, 16, 48.0
    geom = lens.MapGeometry(16, 3.0, (1.0,), c)
    a = np.linspace(0.4, 1.0, 4)
    noise = W.white_noise(np_side, 11)
    rng = np.random.default_rng(12)
    kbar = rng.standard_normal((1, 16, 16))
    return c, np_side, nm, box, geom, a, noise, kbar


def test_full_reverse_pass_matches_finite_difference():
    c, np_side, nm, box, geom, a, noise, kbar = _loss_setup()
    g = adjoint.kappa_vjp_noise(noise, kbar, c, box, nm, a, geom)
    rng = np.random.default_rng(13)
    v = rng.standard_normal(noise.shape)
    eps = 1e-6

    def loss(w):
        k, _ = adjoint.forward_with_checkpoints(w, c, box, nm, a, geom)
        return np.sum(k * kbar)
    fd = (loss(noise + eps * v) - loss(noise - eps * v)) / (2 * eps)
    ad = np.sum(g * v)
    assert abs(fd - ad) < 1e-6 * abs(ad)


def test_sigma8_gradient_is_noise_scaling():
    """The model depends on (sigma8, noise) only through sigma8 * noise, so
    dL/dsigma8 = <dL/dnoise, noise> / sigma8 exactly; checked by central FD."""
    c, np_side, nm, box, geom, a, noise, kbar = _loss_setup()
    g = adjoint.kappa_vjp_noise(noise, kbar, c, box, nm, a, geom)
    ds8 = np.sum(g * noise) / c.sigma8

    def loss(s8):
        cc = Cosmology(0.3, sigma8=s8)
        k, _ = adjoint.forward_with_checkpoints(noise, cc, box, nm, a, geom)
        return np.sum(k * kbar)
    h = 1e-6
    fd = (loss(c.sigma8 + h) - loss(c.sigma8 - h)) / (2 * h)
    assert abs(fd - ds8) < 1e-5 * abs(ds8)


@pytest.mark.parametrize("h", [1e-4, 1e-5])
def test_cosmology_gradients_match_end_to_end_finite_difference(h):
    """Omega_m and sigma_8 cotangents against central differences of the whole
    forward model with the shell partition (chi bounds of the shells) and the
    in-front-of-source test held at the central cosmology: membership is
    piecewise constant and not differentiated (a boundary crossing would
    otherwise put an O(1/h) jump into the difference quotient)."""
    c, np_side, nm, box, geom, a, noise, kbar = _loss_setup()
    nb, g_om, g_s8 = adjoint.kappa_vjp_cosmo(noise, kbar, c, box, nm, a, geom, dom=h)
    ref = adjoint.kappa_vjp_noise(noise, kbar, c, box, nm, a, geom)
    assert np.max(np.abs(nb - ref)) < 1e-12 * np.max(np.abs(ref))
    chis = [c.chi(v) for v in a]

    def loss(om=0.3, s8=0.8):
        cc = Cosmology(om, sigma8=s8)
        gg = lens.MapGeometry(geom.npix, np.degrees(geom.fov), geom.z_src, cc)
        k, _ = adjoint.forward_with_checkpoints(noise, cc, box, nm, a, gg, shell_chis=chis,
                                                src_cut=geom.chi_src)
        return np.sum(k * kbar)
    fd_om = (loss(om=0.3 + h) - loss(om=0.3 - h)) / (2 * h)
    fd_s8 = (loss(s8=0.8 + 1e-6) - loss(s8=0.8 - 1e-6)) / 2e-6
    assert abs(fd_s8 - g_s8) < 1e-5 * abs(g_s8)
    # both sides difference in Omega_m with the same h: they agree to O(h^2)
    assert abs(fd_om - g_om) < 2 * h * abs(g_om)


def test_source_membership_hold_leaves_the_derivative_unchanged():
    """The lens weight is continuous in chi_s (it vanishes at chi = chi_s), so
    holding the in-front-of-source test at the central chi_s must give the
    true derivative.  Shell a 0.4 -> 0.6 straddles the z = 1 source plane and
    holds images 0.005 Mpc in front of it; a step h = 1e-7 in Omega_m moves
    chi_s by 1.4e-4 Mpc and crosses none of them, a step 1e-5 (1.4e-2 Mpc)
    does.  Held membership at 1e-5 must match the free difference at 1e-7."""
    c = Cosmology(0.3)
    geom = lens.MapGeometry(16, 3.0, (1.0,), c)
    a = np.linspace(0.4, 1.0, 4)
    _, states = adjoint.forward_with_checkpoints(W.white_noise(16, 11), c, 48.0, 32, a, geom)
    kbar = np.random.default_rng(12).standard_normal((1, 16, 16))
    x1 = states[1][0]
    cb = (c.chi(a[1]), c.chi(a[0]))

    def d(h, cut):
        vals = []
        for om in (0.3 + h, 0.3 - h):
            cc = Cosmology(om)
            g = lens.MapGeometry(16, 3.0, (1.0,), cc)
            vals.append(np.sum(kbar * lens.project_shell(x1, a[0], a[1], cc, 48.0, 16, g,
                                                         include_mean=False, chi_bounds=cb,
                                                         src_cut=cut)))
        return (vals[0] - vals[1]) / (2 * h)
    ref = d(1e-7, None)
    held = d(1e-5, geom.chi_src)
    free = d(1e-5, None)
    assert abs(held - ref) < 1e-6 * abs(ref)
    assert abs(free - ref) > 1e-4 * abs(ref)     # the kink the hold avoids
