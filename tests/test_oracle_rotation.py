"""Pins of the oracle's replica rotation (the package-design section: the
box is rotated before it is repeated): each replica (nx, ny, nz) is one of
the 48 cube symmetries, chosen by a SplitMix64 hash of its offsets and a
seed."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import adjoint, lens, pm
from oracle.cosmology import Cosmology


def test_mix64_is_splitmix64():
    """The finalizer reproduces the published SplitMix64 sequence for seed
    1234567 (state advanced by the golden-ratio increment)."""
    st, out = 1234567, []
    for _ in range(5):
        st = (st + 0x9E3779B97F4A7C15) & lens._MASK64
        out.append(lens._mix64(st))
    assert out == [6457827717110365317, 3203168211198807973, 9817491932198370423,
                   4593380528125082431, 16408922859458223821]


def test_symmetries_are_48_distinct_bijections_of_the_box():
    box, n = 8.0, 8
    g = (np.arange(n) + 0.5) * box / n
    pts = np.stack(np.meshgrid(g, g, g, indexing="ij")).reshape(3, -1)
    v = np.array([[1.0], [2.0], [3.0]])
    seen = set()
    for s in range(48):
        r = lens.apply_symmetry(pts, s, box)
        # the lattice of cell centres maps onto itself
        key = lambda a: set(map(tuple, np.round(a.T, 9)))
        assert key(r) == key(pts)
        seen.add(tuple(lens.apply_symmetry(v, s)[:, 0]))
    assert len(seen) == 48
    np.testing.assert_array_equal(lens.apply_symmetry(pts, 0, box), pts)


def test_replica_symmetries_spread_over_the_group():
    counts = np.zeros(48, int)
    for nx in range(-6, 7):
        for ny in range(-6, 7):
            for nz in range(0, 12):
                counts[lens.replica_symmetry(nx, ny, nz, 99)] += 1
    assert counts.min() > 0
    # 2028 replicas over 48 symmetries: about 42 each
    assert counts.max() < 3 * counts.mean()
    assert lens.replica_symmetry(1, 2, 3, 5) != lens.replica_symmetry(1, 2, 3, 6) or \
        lens.replica_symmetry(2, 2, 3, 5) != lens.replica_symmetry(2, 2, 3, 6)


def test_symmetric_lattice_is_unchanged_by_rotation(cosmo):
    """The B = 1 lattice of cell centres is invariant under every cube
    symmetry, so its rotated and unrotated projections agree."""
    np_side, box = 12, 150.0
    x = pm.lattice_positions(np_side, np_side, box)
    g0 = lens.MapGeometry(32, 3.0, (1.0, 2.0), cosmo)
    g1 = lens.MapGeometry(32, 3.0, (1.0, 2.0), cosmo, rotation_seed=17)
    k0 = lens.project_shell(x, 0.45, 0.6, cosmo, box, np_side, g0, include_mean=False)
    k1 = lens.project_shell(x, 0.45, 0.6, cosmo, box, np_side, g1, include_mean=False)
    assert np.abs(k0).max() > 0
    assert np.max(np.abs(k1 - k0)) < 1e-10 * np.abs(k0).max()


def test_single_particle_lands_at_its_rotated_image(cosmo):
    """One particle, one replica along the line of sight: the map's centroid
    is the projection of the image under that replica's symmetry."""
    geom = lens.MapGeometry(32, 2.0, (2.0,), cosmo, rotation_seed=3)
    box, np_side = 900.0, 10
    a_far, a_near = 0.6, 0.7
    chi_far, chi_near = cosmo.chi(a_far), cosmo.chi(a_near)
    nz = math.floor(0.5 * (chi_far + chi_near) / box)
    s = lens.replica_symmetry(0, 0, nz, 3)
    # choose the image position, then the box position that maps to it
    img = np.array([0.5 * box + 5.3, 0.5 * box - 7.1, 0.5 * (chi_far + chi_near) - nz * box])
    x = np.empty(3)
    perm, flips = lens.PERMS[s // 8], s % 8
    for j in range(3):
        x[perm[j]] = box - img[j] if flips >> j & 1 else img[j]
    out = lens.project_shell(x[:, None], a_far, a_near, cosmo, box, np_side, geom,
                             include_mean=False)[0]
    assert out.sum() > 0
    chi = img[2] + nz * box
    t = (img[:2] - 0.5 * box) / chi / geom.dtheta + 0.5 * geom.npix - 0.5
    j = np.arange(geom.npix)
    c0 = np.sum(out.sum(axis=1) * j) / out.sum()
    c1 = np.sum(out.sum(axis=0) * j) / out.sum()
    assert abs(c0 - t[0]) < 1e-9 and abs(c1 - t[1]) < 1e-9


def test_rotated_lens_adjoint_matches_finite_difference(cosmo):
    box, np_side = 60.0, 10
    geom = lens.MapGeometry(24, 4.0, (1.0, 1.5), cosmo, rotation_seed=11)
    x = W.clustered_positions(np_side, 20, box, seed=71)
    rng = np.random.default_rng(3)
    kbar = rng.normal(size=(2, 24, 24))
    v = rng.normal(size=x.shape)
    a_far, a_near = 0.45, 0.55
    f = lambda xx: np.sum(kbar * lens.project_shell(xx, a_far, a_near, cosmo, box, np_side,
                                                    geom, include_mean=False))
    h = 1e-6
    fd = (f(x + h * v) - f(x - h * v)) / (2 * h)
    ad = np.sum(adjoint.lens_vjp(x, a_far, a_near, kbar, cosmo, box, np_side, geom) * v)
    assert abs(ad) > 0
    assert abs(ad - fd) < 1e-6 * abs(ad)
