"""Particle-mesh step of FastPM as used by MADLens, float64 (oracle).

Test infrastructure only (see the package header).

What the paper states (package design section): particles start from
Gaussian initial modes, are painted onto a force mesh at B times the
particle-grid resolution, and are stepped with kick and drift factors that
keep linear displacement exact in every step; the initial conditions are
Lagrangian perturbation theory (appendix), here first order (Zel'dovich).
Everything the paper leaves open is fixed as follows:

  mass assignment   cloud-in-cell, mesh node m at position m*H, H = L/Nm
  lattice           particle (i0,i1,i2) sits at q = (B*i + 1/2) * H
  FFT               unnormalised forward transform, inverse carries 1/N^3
  force             f_hat_j = i k_j delta_hat / k^2, zero at k = 0 and on
                    the plane |n_j| = N/2 of component j; no deconvolution
  stepping          kick-drift-kick, one force per step, midpoint
                    a_h = (a_i + a_{i+1}) / 2
  units             x and p in Mpc/h, p = a^3 E dx/da, k in h/Mpc

Pins (tests/test_oracle_pm.py): brute-force DFT on 8^3 and 6^3; the closed
form force of one plane wave; CIC mass conservation, on-node deposit and
exact uniformity of the unperturbed lattice; the paint/readout adjoint
identity; momentum conservation; linear growth of one mode; time
reversibility of the KDK step; the IC spectral identity -i k.s = delta and
the closed-form displacement of a single mode.  The PGD correction
(pgd_displacement) is pinned in tests/test_oracle_pgd.py.
"""
from __future__ import annotations

import numpy as np
import scipy.fft

from .cosmology import Cosmology

FFT_WORKERS = -1  # all host cores


# ---------------------------------------------------------------------------
# lattice and wave numbers
# ---------------------------------------------------------------------------
def lattice_positions(np_side, nm_side, box):
    """q = (B i + 1/2) H per axis for every particle, shape [3][Np^3]."""
    b = nm_side // np_side
    h = box / nm_side
    i = np.indices((np_side,) * 3).reshape(3, -1).astype(np.float64)
    return (b * i + 0.5) * h


def wavenumbers(n, box):
    """k vectors on the rfftn grid of an n^3 mesh, h/Mpc.

    Returns (k0, k1, k2, n0, n1, n2): broadcastable arrays of wave numbers
    and the signed integer mode numbers (fftfreq order, rfftfreq last axis).
    """
    n0 = np.fft.fftfreq(n, d=1.0 / n).round().astype(np.int64)
    n2 = np.fft.rfftfreq(n, d=1.0 / n).round().astype(np.int64)
    kf = 2.0 * np.pi / box
    return (kf * n0[:, None, None], kf * n0[None, :, None], kf * n2[None, None, :],
            n0[:, None, None], n0[None, :, None], n2[None, None, :])


def gradient_inverse_laplacian(field_hat, n, box):
    """Apply i k_j / k^2 to a half spectrum for j = 0, 1, 2.

    The k = 0 mode is zeroed, and component j is zeroed on its Nyquist plane
    |n_j| = n/2, where i k_j has no Hermitian-consistent value.
    """
    k0, k1, k2, n0, n1, n2 = wavenumbers(n, box)
    ksq = k0 ** 2 + k1 ** 2 + k2 ** 2
    ksq_safe = np.where(ksq == 0.0, 1.0, ksq)
    out = []
    for kj, nj in ((k0, n0), (k1, n1), (k2, n2)):
        m = 1j * kj / ksq_safe
        m = np.where(ksq == 0.0, 0.0, m)
        m = np.where(np.abs(nj) == n // 2, 0.0, m)
        out.append(field_hat * m)
    return out


# ---------------------------------------------------------------------------
# initial conditions
# ---------------------------------------------------------------------------
def zeldovich_displacement(noise, cosmo: Cosmology, box):
    """Linear displacement field s (at D = 1) on the particle lattice.

    delta_hat = W sqrt(P(k) Np^3 / L^3) with W = rfftn(noise) and delta_hat(0)=0;
    s_hat_j = i k_j delta_hat / k^2 (Nyquist plane of axis j zeroed);
    s_j = irfftn(s_hat_j).  Returns [3][Np^3] in Mpc/h.
    """
    np_side = noise.shape[0]
    w_hat = scipy.fft.rfftn(noise, workers=FFT_WORKERS)
    k0, k1, k2, *_ = wavenumbers(np_side, box)
    kmag = np.sqrt(k0 ** 2 + k1 ** 2 + k2 ** 2)
    pk = np.where(kmag > 0.0, cosmo.pk_linear(np.where(kmag > 0, kmag, 1.0)), 0.0)
    delta_hat = w_hat * np.sqrt(pk * np_side ** 3 / box ** 3)
    comps = gradient_inverse_laplacian(delta_hat, np_side, box)
    return np.stack([scipy.fft.irfftn(c, s=(np_side,) * 3, workers=FFT_WORKERS)
                     .reshape(-1) for c in comps])


def zeldovich_ic(noise, cosmo: Cosmology, box, nm_side, a0):
    """x0 = q + D(a0) s (wrapped into the box), p0 = g_p(a0) s."""
    np_side = noise.shape[0]
    s = zeldovich_displacement(noise, cosmo, box)
    q = lattice_positions(np_side, nm_side, box)
    x = np.mod(q + cosmo.D(a0) * s, box)
    p = cosmo.gp(a0) * s
    return x, p


# ---------------------------------------------------------------------------
# cloud-in-cell paint and readout
# ---------------------------------------------------------------------------
def cic_weights(x, nm_side, box):
    """Per-axis base node and weights for CIC on an Nm^3 mesh.

    u = (x mod L)/H, i = floor(u), t = u - i; weight 1-t to node i and t to
    node i+1 (both mod Nm).  A u that rounds to Nm wraps to node 0.
    """
    h = box / nm_side
    u = np.mod(x, box) / h
    i = np.floor(u)
    t = u - i
    i = i.astype(np.int64) % nm_side
    return i, t


def _corners(x, nm_side, box):
    i, t = cic_weights(x, nm_side, box)
    for c0 in (0, 1):
        for c1 in (0, 1):
            for c2 in (0, 1):
                c = (c0, c1, c2)
                idx = [(i[d] + c[d]) % nm_side for d in range(3)]
                w = np.ones(x.shape[1])
                for d in range(3):
                    w = w * (t[d] if c[d] else 1.0 - t[d])
                flat = (idx[0] * nm_side + idx[1]) * nm_side + idx[2]
                yield flat, w


def cic_paint(x, nm_side, box, mass=1.0, values=None):
    """Deposit each particle's mass (or `values`) onto the mesh with CIC.

    Returns an Nm^3 array.  With mass = (Nm/Np)^3 the mean is 1.
    """
    out = np.zeros(nm_side ** 3)
    v = mass if values is None else values * mass
    for flat, w in _corners(x, nm_side, box):
        out += np.bincount(flat, weights=w * v, minlength=nm_side ** 3)
    return out.reshape((nm_side,) * 3)


def cic_readout(x, mesh, box):
    """Interpolate a mesh at the particles with the CIC weights of paint."""
    nm_side = mesh.shape[0]
    flatmesh = mesh.reshape(-1)
    out = np.zeros(x.shape[1])
    for flat, w in _corners(x, nm_side, box):
        out += w * flatmesh[flat]
    return out


def density(x, np_side, nm_side, box):
    """rho = (Nm/Np)^3 sum_p W_CIC: mean 1 on the mesh."""
    return cic_paint(x, nm_side, box, mass=(nm_side / np_side) ** 3)


def force_mesh(rho, box):
    """f_j = irfftn(i k_j / k^2 * rfftn(rho - 1)), three real meshes, Mpc/h."""
    n = rho.shape[0]
    d_hat = scipy.fft.rfftn(rho - 1.0, workers=FFT_WORKERS)
    comps = gradient_inverse_laplacian(d_hat, n, box)
    return np.stack([scipy.fft.irfftn(c, s=(n,) * 3, workers=FFT_WORKERS)
                     for c in comps])


def particle_force(x, np_side, nm_side, box):
    """Force at the particles: paint, Fourier solve, CIC readout."""
    rho = density(x, np_side, nm_side, box)
    f = force_mesh(rho, box)
    return np.stack([cic_readout(x, f[j], box) for j in range(3)])


# ---------------------------------------------------------------------------
# PGD correction (the package-design section's first technique)
# ---------------------------------------------------------------------------
def pgd_filter(k, k_l, k_s):
    """O_l(k) O_s(k) = exp(-k_l^2 / k^2) exp(-(k / k_s)^4), zero at k = 0.

    The paper names the technique and its parameters (k_l, k_s, alpha0, mu)
    and defers the operator to its PGD reference; this is that operator as
    read here: a high-pass O_l removing the scales that the PM solver gets
    right and a low-pass O_s removing the noise below the mesh scale.
    """
    k = np.asarray(k, dtype=np.float64)
    ks = np.where(k > 0.0, k, 1.0)
    return np.where(k > 0.0, np.exp(-(k_l / ks) ** 2) * np.exp(-(ks / k_s) ** 4), 0.0)


def pgd_displacement(x, np_side, nm_side, box, alpha, k_l, k_s):
    """S = alpha R(x, IFFT(O_l O_s i k delta_hat / k^2)), [3][N] in Mpc/h.

    The filtered gradient of the potential of the particles' own CIC density
    (the force of force_mesh with the PGD filter), read out at the particles
    with CIC and scaled by alpha = alpha0 a^mu (the caller's).
    """
    rho = density(x, np_side, nm_side, box)
    d_hat = scipy.fft.rfftn(rho - 1.0, workers=FFT_WORKERS)
    k0, k1, k2, *_ = wavenumbers(nm_side, box)
    o = pgd_filter(np.sqrt(k0 ** 2 + k1 ** 2 + k2 ** 2), k_l, k_s)
    comps = gradient_inverse_laplacian(d_hat * o, nm_side, box)
    f = [scipy.fft.irfftn(c, s=(nm_side,) * 3, workers=FFT_WORKERS) for c in comps]
    return alpha * np.stack([cic_readout(x, f[j], box) for j in range(3)])


# ---------------------------------------------------------------------------
# time stepping
# ---------------------------------------------------------------------------
def kdk_step(x, p, f, a0, a1, cosmo: Cosmology, np_side, nm_side, box,
             drift_momentum=False):
    """One kick-drift-kick step a0 -> a1 with force f = f(x) given at a0.

    p += K(a0, ah; a0) f;  x += Dr(a0, a1; ah) p;  f' = f(x);
    p += K(ah, a1; a1) f'.  Returns (x, p, f'), and with `drift_momentum`
    also the momentum the drift used.
    """
    ah = 0.5 * (a0 + a1)
    p = p + cosmo.kick_factor(a0, ah, a0) * f
    p_h = p
    x = np.mod(x + cosmo.drift_factor(a0, a1, ah) * p, box)
    f = particle_force(x, np_side, nm_side, box)
    p = p + cosmo.kick_factor(ah, a1, a1) * f
    if drift_momentum:
        return x, p, f, p_h
    return x, p, f


def run_pm(noise, cosmo: Cosmology, box, nm_side, a_grid, callback=None,
           drift_momentum=False):
    """Zel'dovich ICs at a_grid[0], then one KDK step per interval.

    `callback(i, x, p)` is called after each step with the state at
    a_grid[i+1] (`callback(i, x, p, p_h)` with `drift_momentum`, p_h being
    the momentum of the step's drift).  Returns the final (x, p).
    """
    np_side = noise.shape[0]
    x, p = zeldovich_ic(noise, cosmo, box, nm_side, a_grid[0])
    f = particle_force(x, np_side, nm_side, box)
    for i in range(len(a_grid) - 1):
        x, p, f, p_h = kdk_step(x, p, f, a_grid[i], a_grid[i + 1], cosmo,
                                np_side, nm_side, box, drift_momentum=True)
        if callback is not None:
            if drift_momentum:
                callback(i, x, p, p_h)
            else:
                callback(i, x, p)
    return x, p
