"""Pins of the oracle's sub-evolution projection (the package-design
section's sub-evolution step): an image keeps the shell of its end-of-step
depth and is moved along its step's drift, x(a) = x(a_near) +
Dr(a_near, a; a_h) p_h, to a_p = a(chi_e) before projection."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import adjoint, lens, pm
from oracle.cosmology import Cosmology


@pytest.fixture(scope="module")
def geom(cosmo):
    return lens.MapGeometry(48, 3.0, (1.0, 2.0), cosmo)


@pytest.mark.parametrize("om", [0.25, 0.3, 0.35])
def test_growth_vectorised_matches_quadrature(om):
    c = Cosmology(om)
    a = np.array([0.01, 0.03, 0.1, 0.25, 0.5, 0.8, 1.0, 1.3])
    ref = np.array([c.D(v) for v in a])
    assert np.max(np.abs(c.D_vec(a) / ref - 1.0)) < 1e-13
    # growing mode: D ~ a at early times in this normalisation's units
    assert abs(c.D_vec(1e-4) / c.D_vec(2e-4) - 0.5) < 1e-6


def test_zero_drift_momentum_is_the_plain_projection(cosmo, geom):
    box, np_side = 180.0, 14
    x = W.random_positions(np_side ** 3, box, seed=21)
    a_far, a_near = 0.45, 0.5
    plain = lens.project_shell(x, a_far, a_near, cosmo, box, np_side, geom)
    sub = lens.project_shell(x, a_far, a_near, cosmo, box, np_side, geom,
                             sub=(np.zeros_like(x), 0.5 * (a_far + a_near)))
    np.testing.assert_array_equal(sub, plain)


def test_moved_image_is_the_drift_path_from_the_step_start(cosmo, geom):
    """The image projected with sub-evolution from the end of the step is the
    one the step's own drift reaches at a(chi_e), computed here from the
    start of the step instead: x_s + Dr(a_far, a_p; a_h) p_h."""
    box, np_side = 3000.0, 10       # one replica along the line of sight
    a_far, a_near = 0.5, 0.56
    a_h = 0.5 * (a_far + a_near)
    chi_far, chi_near = cosmo.chi(a_far), cosmo.chi(a_near)
    rng = np.random.default_rng(5)
    n = 40
    # images well inside the shell, near the line of sight
    depth = chi_near + (chi_far - chi_near) * rng.uniform(0.3, 0.7, n)
    th = rng.uniform(-0.35, 0.35, (2, n)) * geom.fov
    p_h = rng.normal(0.0, 400.0, (3, n))   # Mpc/h per unit of the drift factor
    x_e = np.stack([0.5 * box + th[0] * depth, 0.5 * box + th[1] * depth, depth])
    dr_step = cosmo.drift_factor(a_far, a_near, a_h)
    x_s = x_e - dr_step * p_h
    a_p = np.array([cosmo.a_of_chi(c) for c in x_e[2]])
    y = np.stack([x_s[:, i] + cosmo.drift_factor(a_far, a_p[i], a_h) * p_h[:, i]
                  for i in range(n)], axis=1)
    # the moved depths stay inside the shell, so plain membership agrees
    assert np.all((y[2] > chi_near) & (y[2] <= chi_far))
    assert np.max(np.abs(y - x_e)) > 1.0      # the move is not negligible
    sub = lens.project_shell(x_e, a_far, a_near, cosmo, box, np_side, geom,
                             include_mean=False, sub=(p_h, a_h))
    ref = lens.project_shell(y, a_far, a_near, cosmo, box, np_side, geom,
                             include_mean=False)
    assert np.abs(ref).max() > 0
    assert np.max(np.abs(sub - ref)) < 1e-10 * np.abs(ref).max()


def test_run_hands_out_the_drift_momentum(cosmo):
    """The momentum given to the projection is the one the drift used:
    x_{i+1} - x_i = Dr(a_i, a_{i+1}; a_h) p_h (modulo the box)."""
    np_side, nm, box = 8, 8, 64.0
    noise = W.white_noise(np_side, 3)
    a_grid = np.linspace(0.2, 1.0, 4)
    xs = [pm.zeldovich_ic(noise, cosmo, box, nm, a_grid[0])[0]]
    seen = []

    def cb(i, x, p, p_h):
        dr = cosmo.drift_factor(a_grid[i], a_grid[i + 1], 0.5 * (a_grid[i] + a_grid[i + 1]))
        d = np.mod(x - xs[-1] - dr * p_h + 0.5 * box, box) - 0.5 * box
        seen.append(np.abs(d).max())
        xs.append(x.copy())

    pm.run_pm(noise, cosmo, box, nm, a_grid, callback=cb, drift_momentum=True)
    assert len(seen) == 3 and max(seen) < 1e-9


def test_run_with_interpolation_differs_and_keeps_the_mean(cosmo):
    """Sub-evolution changes the maps (the particles move) but not the
    per-shell mean terms, which do not depend on the particles."""
    wl = W.CFG1
    c = Cosmology(wl.omega_m)
    g = lens.MapGeometry(24, 3.0, (1.0,), c)
    noise = W.white_noise(8, 11)
    a_grid = np.linspace(0.3, 1.0, 4)
    k0, _, _ = lens.run_lensing(noise, c, 40.0, 8, a_grid, g)
    k1, _, _ = lens.run_lensing(noise, c, 40.0, 8, a_grid, g, interpolation=True)
    diff = np.abs(k1 - k0).max()
    assert diff > 1e-6 * np.abs(k0).max()
    # every image still lands once: the totals differ only through the
    # weights of moved images (a small relative change)
    assert abs(k1.sum() - k0.sum()) < 0.05 * np.abs(k0).sum()


# ---------------------------------------------------------------------------
# reverse pass with sub-evolution
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("om", [0.25, 0.3])
def test_growth_derivative_vectorised(om):
    c = Cosmology(om)
    a = np.array([0.05, 0.2, 0.5, 0.9, 1.0])
    ref = np.array([c.dD_da(v) for v in a])
    assert np.max(np.abs(c.dD_da_vec(a) / ref - 1.0)) < 1e-12
    h = 1e-5
    fd = (c.D_vec(a + h) - c.D_vec(a - h)) / (2 * h)
    assert np.max(np.abs(fd / ref - 1.0)) < 1e-8


@pytest.mark.parametrize("seed", [None, 13], ids=["plain", "rotated"])
def test_lens_adjoint_with_subevolution_matches_finite_differences(cosmo, seed):
    """Position and drift-momentum cotangents of a sub-evolved shell against
    central differences of the projection (two source planes, one of them
    inside the shell)."""
    box, np_side = 60.0, 10
    geom = lens.MapGeometry(24, 4.0, (1.0, 1.5), cosmo, rotation_seed=seed)
    x = W.clustered_positions(np_side, 20, box, seed=81)
    rng = np.random.default_rng(82)
    p_h = 40.0 * rng.standard_normal(x.shape)
    kbar = rng.standard_normal((2, 24, 24))
    v, u = rng.standard_normal(x.shape), rng.standard_normal(x.shape)
    a_far, a_near = 0.45, 0.55
    a_h = 0.5 * (a_far + a_near)
    f = lambda xx, pp: np.sum(kbar * lens.project_shell(xx, a_far, a_near, cosmo, box, np_side,
                                                        geom, include_mean=False,
                                                        sub=(pp, a_h)))
    xb, pb = adjoint.lens_vjp(x, a_far, a_near, kbar, cosmo, box, np_side, geom, sub=(p_h, a_h))
    # the bilinear weights have kinks at pixel edges; with the rotated
    # replicas' ~1e4 images a step of 1e-6 already straddles some of them
    # (1.5e-4 off), a step of 1e-7 none
    h = 1e-7
    fdx = (f(x + h * v, p_h) - f(x - h * v, p_h)) / (2 * h)
    fdp = (f(x, p_h + h * u) - f(x, p_h - h * u)) / (2 * h)
    adx, adp = np.sum(xb * v), np.sum(pb * u)
    assert abs(adx) > 0 and abs(adp) > 0
    assert abs(adx - fdx) < 1e-6 * abs(adx)
    assert abs(adp - fdp) < 1e-6 * abs(adp)
    # zero drift momentum gives the plain position cotangent (p_h_bar = dr g
    # remains: the move is linear in p_h)
    xb0, _ = adjoint.lens_vjp(x, a_far, a_near, kbar, cosmo, box, np_side, geom,
                              sub=(np.zeros_like(x), a_h))
    plain = adjoint.lens_vjp(x, a_far, a_near, kbar, cosmo, box, np_side, geom)
    assert np.max(np.abs(xb0 - plain)) < 1e-12 * np.abs(plain).max()


def _interp_setup():
    c = Cosmology(0.3)
    geom = lens.MapGeometry(16, 3.0, (1.0,), c)
    a = np.linspace(0.4, 1.0, 4)
    return c, 8, 16, 48.0, geom, a, W.white_noise(8, 11), \
        np.random.default_rng(12).standard_normal((1, 16, 16))


def test_reverse_pass_with_subevolution_matches_finite_difference():
    c, np_side, nm, box, geom, a, noise, kbar = _interp_setup()
    g = adjoint.kappa_vjp_noise(noise, kbar, c, box, nm, a, geom, interpolation=True)
    v = np.random.default_rng(13).standard_normal(noise.shape)
    eps = 1e-6

    def loss(w):
        k, _ = adjoint.forward_with_checkpoints(w, c, box, nm, a, geom, interpolation=True)
        return np.sum(k * kbar)
    fd = (loss(noise + eps * v) - loss(noise - eps * v)) / (2 * eps)
    ad = np.sum(g * v)
    plain = np.sum(adjoint.kappa_vjp_noise(noise, kbar, c, box, nm, a, geom) * v)
    assert abs(fd - ad) < 1e-6 * abs(ad)
    assert abs(plain - ad) > 1e-3 * abs(ad)          # sub-evolution changes the gradient


def test_cosmology_gradients_with_subevolution_match_finite_differences():
    c, np_side, nm, box, geom, a, noise, kbar = _interp_setup()
    h = 1e-5
    nb, g_om, g_s8 = adjoint.kappa_vjp_cosmo(noise, kbar, c, box, nm, a, geom, dom=h,
                                             interpolation=True)
    chis = [c.chi(v) for v in a]

    def loss(om=0.3, s8=0.8):
        cc = Cosmology(om, sigma8=s8)
        gg = lens.MapGeometry(geom.npix, np.degrees(geom.fov), geom.z_src, cc)
        k, _ = adjoint.forward_with_checkpoints(noise, cc, box, nm, a, gg, shell_chis=chis,
                                                src_cut=geom.chi_src, interpolation=True,
                                                hold=c)
        return np.sum(k * kbar)
    fd_om = (loss(om=0.3 + h) - loss(om=0.3 - h)) / (2 * h)
    fd_s8 = (loss(s8=0.8 + 1e-6) - loss(s8=0.8 - 1e-6)) / 2e-6
    assert abs(fd_s8 - g_s8) < 1e-5 * abs(g_s8)
    assert abs(fd_om - g_om) < 2 * h * abs(g_om)


def test_held_membership_of_moved_images(cosmo):
    """With sub-evolution an image's depth moves with Omega_m, so it can cross
    a source plane within a difference step.  One image, moved along the line
    of sight to 1e-6 Mpc/h in front of the z = 1 plane: holding the source
    test at the central cosmology's moved depth gives, at h = 1e-5, the
    derivative that an unheld difference gives at h = 1e-8 (where the image
    stays in front), while the unheld difference at h = 1e-5 puts it behind
    the plane on one side."""
    geom = lens.MapGeometry(32, 2.0, (1.0,), cosmo)
    box, np_side = 900.0, 10
    a_far, a_near = 0.45, 0.55
    ah = 0.5 * (a_far + a_near)
    chis = geom.chi_src[0]
    nz = math.floor(chis / box)
    chi_e = chis + 2.0                       # behind the plane before the move
    dr = (cosmo.D(cosmo.a_of_chi(chi_e)) - cosmo.D(a_near)) / cosmo.gp(ah)
    pz = (-2.0 - 1e-6) / dr                  # moved to chi_s - 1e-6
    # a quarter pixel off the map centre, no transverse momentum
    off = 0.25 * geom.dtheta * chis
    x = np.array([[0.5 * box + off], [0.5 * box - off], [chi_e - nz * box]])
    ph = np.array([[0.0], [0.0], [pz]])
    kbar = np.ones((1, 32, 32))
    cb = (cosmo.chi(a_near), cosmo.chi(a_far))

    def d(h, held):
        vals = []
        for om in (0.3 + h, 0.3 - h):
            cc = Cosmology(om)
            g = lens.MapGeometry(32, 2.0, (1.0,), cc)
            vals.append(np.sum(kbar * lens.project_shell(
                x, a_far, a_near, cc, box, np_side, g, include_mean=False, chi_bounds=cb,
                src_cut=geom.chi_src, sub=(ph, ah), hold=cosmo if held else None)))
        return (vals[0] - vals[1]) / (2 * h)
    k0 = np.sum(lens.project_shell(x, a_far, a_near, cosmo, box, np_side, geom,
                                   include_mean=False, sub=(ph, ah)))
    assert k0 > 0                                # in front of the plane, on the map
    ref = d(1e-8, False)
    assert abs(d(1e-5, True) - ref) < 1e-4 * abs(ref)
    assert abs(d(1e-5, False) - ref) > 1e-2 * abs(ref)
