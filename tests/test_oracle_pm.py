"""Pins of the oracle's particle-mesh step.

Brute-force DFT, closed-form plane-wave force, exact CIC invariants,
adjoint identities, conservation laws, linear growth, reversibility and
the closed-form displacement of a single initial mode.
"""
import itertools
import math

import numpy as np
import pytest
import scipy.fft

import workloads as W
from oracle import pm
from oracle.cosmology import Cosmology


def _brute_rfftn(x):
    n = x.shape[0]
    out = np.zeros((n, n, n // 2 + 1), dtype=np.complex128)
    idx = np.arange(n)
    for k0, k1, k2 in itertools.product(range(n), range(n), range(n // 2 + 1)):
        ph = np.exp(-2j * np.pi * (k0 * idx[:, None, None] + k1 * idx[None, :, None]
                                   + k2 * idx[None, None, :]) / n)
        out[k0, k1, k2] = np.sum(x * ph)
    return out


@pytest.mark.parametrize("n", [8, 6])
def test_fft_matches_brute_force_dft(n):
    rng = np.random.default_rng(3)
    x = rng.standard_normal((n, n, n))
    ref = _brute_rfftn(x)
    got = scipy.fft.rfftn(x)
    assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref))
    back = scipy.fft.irfftn(got, s=x.shape)
    assert np.max(np.abs(back - x)) < 1e-13


@pytest.mark.parametrize("mode", [(1, 0, 0), (2, -3, 1), (0, 5, 7), (3, 3, -2)])
def test_plane_wave_force_closed_form(mode):
    """delta = A cos(k.x) on the mesh nodes gives f = -A k sin(k.x) / k^2."""
    n, box, amp = 16, 50.0, 0.3
    m = np.indices((n,) * 3).astype(np.float64) * (box / n)
    kv = [2 * np.pi * mi / box for mi in mode]
    ph = kv[0] * m[0] + kv[1] * m[1] + kv[2] * m[2]
    rho = 1.0 + amp * np.cos(ph)
    f = pm.force_mesh(rho, box)
    ksq = sum(k * k for k in kv)
    for j in range(3):
        exact = -amp * kv[j] / ksq * np.sin(ph)
        assert np.max(np.abs(f[j] - exact)) < 1e-13


def test_force_zero_mean_and_nyquist_plane():
    rng = np.random.default_rng(5)
    rho = 1.0 + 0.1 * rng.standard_normal((8, 8, 8))
    f = pm.force_mesh(rho, 20.0)
    assert np.max(np.abs(f.sum(axis=(1, 2, 3)))) < 1e-12
    # a mode living only on the Nyquist plane of axis 0 produces no f_0
    m = np.indices((8,) * 3)
    rho = 1.0 + np.cos(np.pi * m[0]) * np.cos(2 * np.pi * m[1] / 8)
    f = pm.force_mesh(rho, 20.0)
    assert np.max(np.abs(f[0])) < 1e-14
    assert np.max(np.abs(f[1])) > 1e-2


def test_repeated_configuration_has_the_force_of_one_copy():
    """A configuration repeated 2 x 2 x 2 in a box twice as large (same cell
    size) has, node for node and particle for particle, the density and
    force of one copy: its transform lives on even modes, where the doubled
    box's wave numbers equal the original's (and its Nyquist planes are the
    original's)."""
    L, np_s, nm_s = 40.0, 16, 32
    n = np_s ** 3
    x = W.clustered_positions(np_s, nm_s, L, seed=66)
    offs = [np.array([(c >> 2) & 1, (c >> 1) & 1, c & 1])[:, None] * L for c in range(8)]
    xb = np.concatenate([x + o for o in offs], axis=1)
    f = pm.force_mesh(pm.density(x, np_s, nm_s, L), L)
    fb = pm.force_mesh(pm.density(xb, 2 * np_s, 2 * nm_s, 2 * L), 2 * L)
    for c in range(8):
        i, j, k = ((c >> 2) & 1) * nm_s, ((c >> 1) & 1) * nm_s, (c & 1) * nm_s
        assert np.max(np.abs(fb[:, i:i + nm_s, j:j + nm_s, k:k + nm_s] - f)) <= 1e-12 * np.max(np.abs(f))
    a = pm.particle_force(x, np_s, nm_s, L)
    ab = pm.particle_force(xb, 2 * np_s, 2 * nm_s, 2 * L)
    for c in range(8):
        assert np.max(np.abs(ab[:, c * n:(c + 1) * n] - a)) <= 1e-12 * np.max(np.abs(a))


def test_paint_mass_conservation():
    x = W.random_positions(5000, 37.0, seed=11)
    rho = pm.density(x, 17, 12, 37.0)  # 17^3 = 4913 < 5000: mass per particle
    np_side, nm = 17, 12
    assert abs(rho.sum() - 5000 * (nm / np_side) ** 3) < 1e-9


def test_paint_on_node_single_cell():
    n, box = 8, 16.0
    x = np.array([[3 * 2.0], [5 * 2.0], [7 * 2.0]])
    rho = pm.cic_paint(x, n, box)
    assert rho[3, 5, 7] == 1.0
    assert rho.sum() == 1.0


@pytest.mark.parametrize("np_side,nm", [(8, 8), (8, 16), (6, 12)])
def test_unperturbed_lattice_is_exactly_uniform(np_side, nm):
    q = pm.lattice_positions(np_side, nm, 30.0)
    rho = pm.density(q, np_side, nm, 30.0)
    assert np.all(rho == 1.0)


def test_paint_shift_commutes():
    n, box = 8, 24.0
    x = W.random_positions(300, box, seed=2)
    shift = np.array([2, -3, 5])
    rho = pm.cic_paint(x, n, box)
    rho_s = pm.cic_paint(np.mod(x + (shift * box / n)[:, None], box), n, box)
    assert np.max(np.abs(rho_s - np.roll(rho, tuple(shift), axis=(0, 1, 2)))) < 1e-12


def test_paint_readout_adjoint_identity():
    n, box = 9, 13.0
    rng = np.random.default_rng(1)
    x = W.random_positions(400, box, seed=3)
    v = rng.standard_normal(400)
    y = rng.standard_normal((n, n, n))
    lhs = np.sum(pm.cic_paint(x, n, box, values=v) * y)
    rhs = np.sum(v * pm.cic_readout(x, y, box))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_readout_reproduces_linear_field_inside_cells():
    n, box = 10, 10.0
    m = np.indices((n,) * 3).astype(np.float64)
    field = 0.5 + 1.5 * m[0] - 0.25 * m[1] + 2.0 * m[2]
    rng = np.random.default_rng(4)
    x = rng.uniform(1.0, 8.0, size=(3, 200))  # away from the periodic seam
    got = pm.cic_readout(x, field, box)
    exact = 0.5 + 1.5 * x[0] - 0.25 * x[1] + 2.0 * x[2]
    assert np.max(np.abs(got - exact)) < 1e-12


def test_momentum_conservation_of_pm_force():
    x = W.clustered_positions(8, 16, 40.0, seed=9)
    f = pm.particle_force(x, 8, 16, 40.0)
    assert np.max(np.abs(f.sum(axis=1))) < 1e-11 * np.abs(f).sum()


def test_ic_spectral_identity(cosmo):
    np_side, box = 16, 64.0
    noise = W.white_noise(np_side, 21)
    s = pm.zeldovich_displacement(noise, cosmo, box)
    k0, k1, k2, n0, n1, n2 = pm.wavenumbers(np_side, box)
    div = sum(-1j * kj * scipy.fft.rfftn(s[j].reshape((np_side,) * 3))
              for j, kj in enumerate((k0, k1, k2)))
    kmag = np.sqrt(k0 ** 2 + k1 ** 2 + k2 ** 2)
    pk = np.where(kmag > 0, cosmo.pk_linear(np.where(kmag > 0, kmag, 1.0)), 0.0)
    delta_hat = scipy.fft.rfftn(noise) * np.sqrt(pk * np_side ** 3 / box ** 3)
    ok = (np.abs(n0) != np_side // 2) & (np.abs(n1) != np_side // 2) \
        & (np.abs(n2) != np_side // 2)
    ok = np.broadcast_to(ok, div.shape)
    assert np.max(np.abs(div - delta_hat)[ok]) < 1e-10 * np.max(np.abs(delta_hat))


@pytest.mark.parametrize("mode", [(1, 2, 0), (0, 3, 5), (4, -1, 2)])
def test_ic_single_mode_closed_form(cosmo, mode):
    """w = cos(2 pi n.i/N) gives s_j(i) = -k_j/k^2 sqrt(P N^3/L^3) sin(2 pi n.i/N)."""
    np_side, box = 16, 80.0
    noise = W.single_mode_noise(np_side, mode)
    s = pm.zeldovich_displacement(noise, cosmo, box)
    i = np.indices((np_side,) * 3).reshape(3, -1).astype(np.float64)
    ph = 2 * np.pi * (mode[0] * i[0] + mode[1] * i[1] + mode[2] * i[2]) / np_side
    kv = [2 * np.pi * m / box for m in mode]
    k = math.sqrt(sum(v * v for v in kv))
    amp = math.sqrt(float(cosmo.pk_linear(k)) * np_side ** 3 / box ** 3)
    for j in range(3):
        exact = -kv[j] / k ** 2 * amp * np.sin(ph)
        assert np.max(np.abs(s[j] - exact)) < 1e-10 * amp / k


def test_zero_noise_stays_static(cosmo):
    np_side, nm, box = 8, 16, 40.0
    noise = np.zeros((np_side,) * 3)
    x, p = pm.run_pm(noise, cosmo, box, nm, np.linspace(0.1, 1.0, 4))
    q = pm.lattice_positions(np_side, nm, box)
    assert np.max(np.abs(x - q)) < 1e-12
    assert np.max(np.abs(p)) < 1e-12


def test_kdk_time_reversible(cosmo):
    np_side, nm, box = 8, 16, 40.0
    noise = W.white_noise(np_side, 5)
    a0, a1 = 0.3, 0.45
    x0, p0 = pm.zeldovich_ic(noise, cosmo, box, nm, a0)
    f0 = pm.particle_force(x0, np_side, nm, box)
    x1, p1, f1 = pm.kdk_step(x0, p0, f0, a0, a1, cosmo, np_side, nm, box)
    x2, p2, _ = pm.kdk_step(x1, p1, f1, a1, a0, cosmo, np_side, nm, box)
    dx = np.mod(x2 - x0 + 0.5 * box, box) - 0.5 * box
    assert np.max(np.abs(dx)) < 1e-12 * box
    assert np.max(np.abs(p2 - p0)) < 1e-12 * np.max(np.abs(p0))


def test_total_momentum_conserved(cosmo):
    np_side, nm, box = 8, 16, 40.0
    noise = W.white_noise(np_side, 6)
    moms = []
    pm.run_pm(noise, cosmo, box, nm, np.linspace(0.05, 1.0, 6),
              callback=lambda i, x, p: moms.append(p.sum(axis=1)))
    scale = np_side ** 3 * 1e-2
    assert np.max(np.abs(np.array(moms))) < 1e-12 * scale


def test_linear_growth_of_one_mode():
    """A small single mode grows as D(a)/D(a0) through the KDK steps.

    The PM force of a mode is short of the exact one by the CIC windows
    (paint and readout), about (kH)^2/6 = 0.16% on a 64^3 mesh for the
    fundamental; the growth error stays below 1%.
    """
    c = Cosmology(0.3)
    np_side, nm, box = 64, 64, 100.0
    mode = (1, 0, 0)
    noise = 1e-6 * W.single_mode_noise(np_side, mode)
    a_grid = np.linspace(0.1, 1.0, 11)
    s = pm.zeldovich_displacement(noise, c, box)
    x, p = pm.run_pm(noise, c, box, nm, a_grid)
    q = pm.lattice_positions(np_side, nm, box)
    disp = np.mod(x - q + 0.5 * box, box) - 0.5 * box
    ratio = np.sum(disp[0] * s[0]) / np.sum(s[0] * s[0])
    assert abs(ratio / (c.D(1.0)) - 1.0) < 0.01
    ratio_p = np.sum(p[0] * s[0]) / np.sum(s[0] * s[0])
    assert abs(ratio_p / c.gp(1.0) - 1.0) < 0.01
