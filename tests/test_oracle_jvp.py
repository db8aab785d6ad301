"""Pins of the oracle's forward-mode tangents (oracle/jvp.py): central finite
differences of the forward oracle, as in the paper's derivative checks (one
perturbed initial-condition pixel, sigma_8, Omega_m with single-mode initial
conditions), and the transpose identity <kbar, J v> = <J^T kbar, v> against
the reverse pass (itself pinned by finite differences)."""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint, jvp, lens, pm
from oracle.cosmology import Cosmology


def test_tangent_paint_matches_finite_difference():
    np_side, nm, box = 8, 16, 40.0
    x = W.clustered_positions(np_side, nm, box, seed=31)
    v = np.random.default_rng(32).standard_normal(x.shape)
    mass = (nm / np_side) ** 3
    h = 1e-6
    fd = (pm.cic_paint(np.mod(x + h * v, box), nm, box, mass)
          - pm.cic_paint(np.mod(x - h * v, box), nm, box, mass)) / (2 * h)
    an = jvp.cic_paint_tangent(x, v, nm, box, mass)
    assert np.abs(an).max() > 0
    # piecewise linear in x: exact unless a particle crosses a cell face
    assert np.max(np.abs(fd - an)) < 1e-6 * np.abs(an).max()
    # total mass is conserved along any direction
    assert abs(an.sum()) < 1e-10 * np.abs(an).max() * an.size


def test_force_jvp_matches_finite_difference_and_transposes_the_vjp():
    np_side, nm, box = 8, 16, 40.0
    x = W.clustered_positions(np_side, nm, box, seed=33)
    rng = np.random.default_rng(34)
    v = rng.standard_normal(x.shape)
    fbar = rng.standard_normal(x.shape)
    h = 1e-6
    fd = (pm.particle_force(np.mod(x + h * v, box), np_side, nm, box)
          - pm.particle_force(np.mod(x - h * v, box), np_side, nm, box)) / (2 * h)
    an = jvp.force_jvp(x, v, np_side, nm, box)
    assert np.max(np.abs(fd - an)) < 1e-6 * np.abs(an).max()
    lhs = np.sum(fbar * an)
    rhs = np.sum(adjoint.force_vjp(x, fbar, np_side, nm, box) * v)
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)


@pytest.mark.parametrize("seed", [None, 11], ids=["plain", "rotated"])
def test_lens_jvp_matches_finite_difference_and_transposes_the_vjp(cosmo, seed):
    box, np_side = 60.0, 10
    geom = lens.MapGeometry(24, 4.0, (1.0, 1.5), cosmo, rotation_seed=seed)
    x = W.clustered_positions(np_side, 20, box, seed=35)
    rng = np.random.default_rng(36)
    v = rng.standard_normal(x.shape)
    kbar = rng.standard_normal((2, 24, 24))
    a_far, a_near = 0.45, 0.55
    proj = lambda xx: lens.project_shell(xx, a_far, a_near, cosmo, box, np_side, geom,
                                         include_mean=False)
    h = 1e-6
    fd = (proj(x + h * v) - proj(x - h * v)) / (2 * h)
    an = jvp.lens_jvp(x, v, a_far, a_near, cosmo, box, np_side, geom)
    assert np.abs(an).max() > 0
    assert np.sqrt(np.mean((fd - an) ** 2)) < 1e-6 * np.sqrt(np.mean(an ** 2))
    lhs = np.sum(kbar * an)
    rhs = np.sum(adjoint.lens_vjp(x, a_far, a_near, kbar, cosmo, box, np_side, geom) * v)
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)


def _setup(seed=None):
    c = Cosmology(0.3)
    np_side, nm, box = 8, 16, 48.0
    geom = lens.MapGeometry(16, 3.0, (1.0, 2.0), c, rotation_seed=seed)
    a = np.linspace(0.4, 1.0, 4)
    noise = W.white_noise(np_side, 11)
    return c, np_side, nm, box, geom, a, noise


def test_single_pixel_noise_tangent_matches_finite_difference():
    """The paper's first derivative check: one initial-condition pixel
    perturbed, directional derivative against a central difference."""
    c, np_side, nm, box, geom, a, noise = _setup()
    e = np.zeros_like(noise)
    e[3, 5, 2] = 1.0
    k, kd = jvp.kappa_jvp(noise, e, 0.0, 0.0, c, box, nm, a, geom)
    h = 1e-5
    fd = (jvp.kappa_at(noise + h * e, c, box, nm, a, geom)
          - jvp.kappa_at(noise - h * e, c, box, nm, a, geom)) / (2 * h)
    assert np.abs(kd).max() > 1e-6 * np.abs(k).max()
    assert np.sqrt(np.mean((fd - kd) ** 2)) < 1e-6 * np.sqrt(np.mean(kd ** 2))


def test_sigma8_tangent_matches_finite_difference():
    """sigma_8 scales the noise: its tangent is the noise tangent along
    noise / sigma_8, and matches a central difference of the model."""
    c, np_side, nm, box, geom, a, noise = _setup()
    _, kd = jvp.kappa_jvp(noise, np.zeros_like(noise), 0.0, 1.0, c, box, nm, a, geom)
    _, kn = jvp.kappa_jvp(noise, noise / c.sigma8, 0.0, 0.0, c, box, nm, a, geom)
    assert np.max(np.abs(kd - kn)) < 1e-12 * np.abs(kd).max()
    h = 1e-6
    fd = (jvp.kappa_at(noise, Cosmology(0.3, sigma8=c.sigma8 + h), box, nm, a, geom)
          - jvp.kappa_at(noise, Cosmology(0.3, sigma8=c.sigma8 - h), box, nm, a, geom)) / (2 * h)
    assert np.sqrt(np.mean((fd - kd) ** 2)) < 1e-6 * np.sqrt(np.mean(kd ** 2))


@pytest.mark.parametrize("mode", [(1, 0, 0), (0, 2, 1), (1, 1, 3)])
def test_omega_m_tangent_of_single_mode_ics_matches_finite_difference(mode):
    """The paper's Omega_m check with single-mode initial conditions: the
    tangent against a central difference of the whole model with the shell
    partition and source membership held (both difference the scalar
    factors with the same step, so they agree to O(h^2))."""
    c, np_side, nm, box, geom, a, _ = _setup()
    q = np.indices((np_side,) * 3)
    noise = 4.0 * np.cos(2 * np.pi * sum(m * qq for m, qq in zip(mode, q)) / np_side + 0.3)
    h = 1e-5
    _, kd = jvp.kappa_jvp(noise, np.zeros_like(noise), 1.0, 0.0, c, box, nm, a, geom, dom=h)
    chis = [c.chi(v) for v in a]

    def model(om):
        cc = Cosmology(om)
        gg = lens.MapGeometry(geom.npix, np.degrees(geom.fov), geom.z_src, cc)
        return jvp.kappa_at(noise, cc, box, nm, a, gg, shell_chis=chis, src_cut=geom.chi_src)
    fd = (model(0.3 + h) - model(0.3 - h)) / (2 * h)
    assert np.abs(kd).max() > 0
    assert np.sqrt(np.mean((fd - kd) ** 2)) < 1e-6 * np.sqrt(np.mean(kd ** 2))


@pytest.mark.parametrize("seed", [None, 7], ids=["plain", "rotated"])
def test_jvp_transposes_the_reverse_pass(seed):
    """<kbar, J (v, Om_dot, s8_dot)> = <noise_bar, v> + Om_bar Om_dot +
    s8_bar s8_dot: both passes difference the same scalar factors, so the
    identity holds to round-off."""
    c, np_side, nm, box, geom, a, noise = _setup(seed)
    rng = np.random.default_rng(37)
    v = rng.standard_normal(noise.shape)
    kbar = rng.standard_normal((2, 16, 16))
    om_dot, s8_dot = 0.7, -1.3
    _, kd = jvp.kappa_jvp(noise, v, om_dot, s8_dot, c, box, nm, a, geom)
    nb, g_om, g_s8 = adjoint.kappa_vjp_cosmo(noise, kbar, c, box, nm, a, geom)
    lhs = np.sum(kbar * kd)
    rhs = np.sum(nb * v) + g_om * om_dot + g_s8 * s8_dot
    assert abs(lhs - rhs) < 1e-9 * (abs(np.sum(nb * v)) + abs(g_om * om_dot) + abs(g_s8 * s8_dot))


def test_tangent_is_linear_in_the_direction():
    c, np_side, nm, box, geom, a, noise = _setup()
    rng = np.random.default_rng(38)
    v = rng.standard_normal(noise.shape)
    _, k1 = jvp.kappa_jvp(noise, v, 0.0, 0.0, c, box, nm, a, geom)
    _, k2 = jvp.kappa_jvp(noise, -2.5 * v, 0.0, 0.0, c, box, nm, a, geom)
    _, k3 = jvp.kappa_jvp(noise, np.zeros_like(v), 0.4, 0.0, c, box, nm, a, geom)
    _, k4 = jvp.kappa_jvp(noise, v, 0.4, 0.0, c, box, nm, a, geom)
    scale = np.abs(k4).max()
    assert np.max(np.abs(k2 + 2.5 * k1)) < 1e-12 * scale
    assert np.max(np.abs(k4 - k1 - k3)) < 1e-12 * scale


@pytest.mark.parametrize("seed", [None, 11], ids=["plain", "rotated"])
def test_lens_tangent_with_subevolution(cosmo, seed):
    """Sub-evolved shell: the tangent along (x_dot, p_h_dot) against a central
    difference of the projection (step 1e-7: the bilinear weights' pixel-edge
    kinks), and the transpose identity with the sub-evolved adjoint."""
    box, np_side = 60.0, 10
    geom = lens.MapGeometry(24, 4.0, (1.0, 1.5), cosmo, rotation_seed=seed)
    x = W.clustered_positions(np_side, 20, box, seed=91)
    rng = np.random.default_rng(92)
    p_h = 40.0 * rng.standard_normal(x.shape)
    v, u = rng.standard_normal(x.shape), rng.standard_normal(x.shape)
    kbar = rng.standard_normal((2, 24, 24))
    a_far, a_near = 0.45, 0.55
    a_h = 0.5 * (a_far + a_near)
    proj = lambda xx, pp: lens.project_shell(xx, a_far, a_near, cosmo, box, np_side, geom,
                                             include_mean=False, sub=(pp, a_h))
    h = 1e-7
    fd = (proj(x + h * v, p_h + h * u) - proj(x - h * v, p_h - h * u)) / (2 * h)
    an = jvp.lens_jvp(x, v, a_far, a_near, cosmo, box, np_side, geom, sub=(p_h, a_h), ph_dot=u)
    assert np.abs(an).max() > 0
    assert np.sqrt(np.mean((fd - an) ** 2)) < 1e-6 * np.sqrt(np.mean(an ** 2))
    xb, pb = adjoint.lens_vjp(x, a_far, a_near, kbar, cosmo, box, np_side, geom, sub=(p_h, a_h))
    lhs = np.sum(kbar * an)
    rhs = np.sum(xb * v) + np.sum(pb * u)
    assert abs(lhs - rhs) < 1e-11 * (abs(np.sum(xb * v)) + abs(np.sum(pb * u)))


def test_jvp_with_subevolution_transposes_the_reverse_pass():
    c, np_side, nm, box, geom, a, noise = _setup()
    rng = np.random.default_rng(93)
    v = rng.standard_normal(noise.shape)
    kbar = rng.standard_normal((2, 16, 16))
    om_dot, s8_dot = 0.7, -1.3
    k, kd = jvp.kappa_jvp(noise, v, om_dot, s8_dot, c, box, nm, a, geom, interpolation=True)
    k0, _ = adjoint.forward_with_checkpoints(noise, c, box, nm, a, geom, interpolation=True)
    assert np.max(np.abs(k - k0)) < 1e-12 * np.abs(k0).max()
    nb, g_om, g_s8 = adjoint.kappa_vjp_cosmo(noise, kbar, c, box, nm, a, geom,
                                             interpolation=True)
    lhs = np.sum(kbar * kd)
    rhs = np.sum(nb * v) + g_om * om_dot + g_s8 * s8_dot
    assert abs(lhs - rhs) < 1e-9 * (abs(np.sum(nb * v)) + abs(g_om * om_dot) + abs(g_s8 * s8_dot))
    _, kd_plain = jvp.kappa_jvp(noise, v, om_dot, s8_dot, c, box, nm, a, geom)
    assert np.sqrt(np.mean((kd - kd_plain) ** 2)) > 1e-3 * np.sqrt(np.mean(kd ** 2))
