"""Vector-Jacobian products of the forward model, float64 (oracle).

Test infrastructure only (see the package header).

The paper differentiates MADLens by reverse-mode automatic differentiation
over a recorded tape, with respect to the initial Gaussian modes and, in a
second variant, Omega_m and sigma_8; the cosmology dependence of scalar
factors (initial-condition amplitude, kick and drift factors) is handled by
finite differences of those scalar factors (design section; appendix on
cosmology derivatives).  This module writes the same reverse pass out by
hand:

  force node   f = R(x, M(P(x)))  with P the CIC paint, M the Fourier force
               operator and R the CIC readout.  Its VJP for a cotangent fbar:
                 xbar += dR/dx^T fbar            (CIC gradient gather on M)
                 Mbar  = R_M^T fbar               (paint of fbar, no mass)
                 rhobar = M^T Mbar = sum_j irfftn(conj(m_j) rfftn(Mbar_j))
                 xbar += dP/dx^T rhobar           (CIC gradient gather on rhobar)
               CIC derivative: -1 to node floor(u), +1 to node floor(u)+1 per
               axis (one-sided at integer u, consistent with floor).
  KDK step     ph = p + K1 f(x);  x' = x + Dr ph;  p' = ph + K2 f(x').
  shells       membership and replica choice are piecewise constant and get
               no gradient.

Pins (tests/test_oracle_adjoint.py): central finite differences of the
forward oracle for every VJP, and the dot-product identity for the linear
pieces.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.fft

from . import lens, pm
from .cosmology import Cosmology, lens_prefactor

FFT_WORKERS = -1


# ---------------------------------------------------------------------------
# CIC gradient gather
# ---------------------------------------------------------------------------
def cic_gradient_gather(x, mesh, box):
    """d/dx of the CIC readout of `mesh` at x: [3][N] (per Mpc/h).

    sum over corners of dW/du_d * prod_{e != d} W_e * mesh(corner) / H.
    """
    nm = mesh.shape[0]
    h = box / nm
    i, t = pm.cic_weights(x, nm, box)
    flat_mesh = mesh.reshape(-1)
    out = np.zeros_like(x)
    for c0 in (0, 1):
        for c1 in (0, 1):
            for c2 in (0, 1):
                c = (c0, c1, c2)
                idx = [(i[d] + c[d]) % nm for d in range(3)]
                flat = (idx[0] * nm + idx[1]) * nm + idx[2]
                val = flat_mesh[flat]
                w = [t[d] if c[d] else 1.0 - t[d] for d in range(3)]
                dw = [1.0 if c[d] else -1.0 for d in range(3)]
                out[0] += dw[0] * w[1] * w[2] * val
                out[1] += w[0] * dw[1] * w[2] * val
                out[2] += w[0] * w[1] * dw[2] * val
    return out / h


def force_operator_transpose(mesh_bar, box):
    """rhobar = sum_j irfftn(conj(m_j) rfftn(Mbar_j)), m_j = i k_j/k^2 with
    the Nyquist zeroing of the forward operator."""
    n = mesh_bar.shape[1]
    k0, k1, k2, n0, n1, n2 = pm.wavenumbers(n, box)
    ksq = k0 ** 2 + k1 ** 2 + k2 ** 2
    ksq_safe = np.where(ksq == 0.0, 1.0, ksq)
    acc = 0.0
    for j, (kj, nj) in enumerate(((k0, n0), (k1, n1), (k2, n2))):
        m = 1j * kj / ksq_safe
        m = np.where(ksq == 0.0, 0.0, m)
        m = np.where(np.abs(nj) == n // 2, 0.0, m)
        acc = acc + np.conj(m) * scipy.fft.rfftn(mesh_bar[j], workers=FFT_WORKERS)
    return scipy.fft.irfftn(acc, s=(n,) * 3, workers=FFT_WORKERS)


def force_vjp(x, f_bar, np_side, nm_side, box):
    """Cotangent of positions for f(x) = particle_force(x) and cotangent f_bar."""
    mass = (nm_side / np_side) ** 3
    rho = pm.density(x, np_side, nm_side, box)
    fmesh = pm.force_mesh(rho, box)
    xbar = np.zeros_like(x)
    # readout part: f_j = R(x, M_j)
    for j in range(3):
        xbar += f_bar[j] * cic_gradient_gather(x, fmesh[j], box)
    mesh_bar = np.stack([pm.cic_paint(x, nm_side, box, mass=1.0, values=f_bar[j])
                         for j in range(3)])
    rho_bar = force_operator_transpose(mesh_bar, box)
    # paint part: rho = mass * sum_p W(x_p - m)
    xbar += mass * cic_gradient_gather(x, rho_bar, box)
    return xbar


# ---------------------------------------------------------------------------
# lens projection
# ---------------------------------------------------------------------------
def bilinear_gather_grad(t0, t1, kmap):
    """(value, d/dt0, d/dt1) of the bilinear gather of kmap at (t0, t1)."""
    npix = kmap.shape[0]
    j0 = np.floor(t0).astype(np.int64)
    j1 = np.floor(t1).astype(np.int64)
    f0 = t0 - j0
    f1 = t1 - j1
    v = np.zeros(t0.shape)
    g0 = np.zeros(t0.shape)
    g1 = np.zeros(t0.shape)
    for d0, w0, dw0 in ((0, 1.0 - f0, -1.0), (1, f0, 1.0)):
        for d1, w1, dw1 in ((0, 1.0 - f1, -1.0), (1, f1, 1.0)):
            a = j0 + d0
            b = j1 + d1
            ok = (a >= 0) & (a < npix) & (b >= 0) & (b < npix)
            m = np.zeros(t0.shape)
            m[ok] = kmap[a[ok], b[ok]]
            v += w0 * w1 * m
            g0 += dw0 * w1 * m
            g1 += w0 * dw1 * m
    return v, g0, g1


def lens_vjp(x, a_far, a_near, kappa_bar, cosmo: Cosmology, box, np_side,
             geom: lens.MapGeometry, sub=None):
    """Cotangent of positions for the shell's convergence (particle term).

    Per image: kappa += w(chi) B(t0, t1), t = (r_perp / chi) / dtheta + c,
    w = pref V_p (chi_s - chi) / (chi_s chi a(chi) Omega_pix).

    With `sub` = (p_h, a_h) (sub-evolution, lens.project_shell's `sub`) an
    image at end-of-step depth chi_e is projected at r' = r + dr p_h with
    dr = (D(a(chi_e)) - D(a_near)) / g_p(a_h); with g the gradient of the
    splat at r', the image's cotangents are
      r_bar = g + e_z (d dr / d chi_e) (g . p_h),   p_h_bar = dr g,
    and the call returns (x_bar, p_h_bar).
    """
    chi_far = float(cosmo.chi(a_far))
    chi_near = float(cosmo.chi(a_near))
    pref = lens_prefactor(cosmo.omega_m)
    vp = (box / np_side) ** 3
    xbar = np.zeros_like(x)
    phbar = np.zeros_like(x) if sub is not None else None
    c = 0.5 * geom.npix - 0.5
    if sub is not None:
        p_h, a_h = sub
        d_near, gp_h = cosmo.D(a_near), cosmo.gp(a_h)
    for idx, rx, ry, chi, sym in lens.shell_images(x, box, chi_near, chi_far, geom):
        perm, flips = lens.PERMS[sym // 8], sym % 8
        sgn = [-1.0 if flips >> j & 1 else 1.0 for j in range(3)]
        if sub is not None:
            # the drift momentum in the image frame, and the move along it
            ph = [sgn[j] * p_h[perm[j], idx] for j in range(3)]
            ae = cosmo.a_of_chi_vec(chi)
            dr = (cosmo.D_vec(ae) - d_near) / gp_h
            ddr = cosmo.dD_da_vec(ae) * (-ae * ae * cosmo.E(ae) / 2997.92458) / gp_h
            rx = rx + dr * ph[0]
            ry = ry + dr * ph[1]
            chi = chi + dr * ph[2]
        t0 = rx / chi / geom.dtheta + c
        t1 = ry / chi / geom.dtheta + c
        keep = (t0 > -1.0) & (t0 < geom.npix) & (t1 > -1.0) & (t1 < geom.npix) & (chi > 0.0)
        if not np.any(keep):
            continue
        idx, rx, ry, chi, t0, t1 = idx[keep], rx[keep], ry[keep], chi[keep], t0[keep], t1[keep]
        a = cosmo.a_of_chi_vec(chi)
        dadchi = -a * a * cosmo.E(a) / 2997.92458
        gx, gy, gz = (np.zeros(idx.size) for _ in range(3))
        for s, chis in enumerate(geom.chi_src):
            src = chi < chis
            if not np.any(src):
                continue
            ch, aa, da = chi[src], a[src], dadchi[src]
            g = (chis - ch) / (chis * ch * aa)
            w = pref * vp * g / geom.omega_pix
            dg = -1.0 / (chis * ch * aa) - g / ch - g * da / aa
            dw = pref * vp * dg / geom.omega_pix
            v, g0, g1 = bilinear_gather_grad(t0[src], t1[src], kappa_bar[s])
            inv = 1.0 / (ch * geom.dtheta)
            gx[src] += w * g0 * inv
            gy[src] += w * g1 * inv
            gz[src] += dw * v - w * (g0 * rx[src] + g1 * ry[src]) * inv / ch
        img = [gx, gy, gz]
        if sub is not None:
            ph = [v[keep] for v in ph]
            dr, ddr = dr[keep], ddr[keep]
            img = [gx, gy, gz + ddr * (gx * ph[0] + gy * ph[1] + gz * ph[2])]
            for j, gj in enumerate((gx, gy, gz)):
                np.add.at(phbar[perm[j]], idx, sgn[j] * dr * gj)
        # back from the image frame: image axis j is box axis perm[j]
        for j, gj in enumerate(img):
            np.add.at(xbar[perm[j]], idx, sgn[j] * gj)
    return xbar if sub is None else (xbar, phbar)


# ---------------------------------------------------------------------------
# initial conditions
# ---------------------------------------------------------------------------
def ic_displacement_transpose(s_bar, cosmo: Cosmology, box):
    """noise_bar = sum_j irfftn(conj(i k_j/k^2) sqrt(P N^3/L^3) rfftn(sbar_j))."""
    np_side = s_bar.shape[1] if s_bar.ndim == 4 else round(s_bar.shape[1] ** (1 / 3))
    sb = s_bar.reshape(3, np_side, np_side, np_side)
    k0, k1, k2, n0, n1, n2 = pm.wavenumbers(np_side, box)
    ksq = k0 ** 2 + k1 ** 2 + k2 ** 2
    kmag = np.sqrt(ksq)
    pk = np.where(kmag > 0.0, cosmo.pk_linear(np.where(kmag > 0, kmag, 1.0)), 0.0)
    amp = np.sqrt(pk * np_side ** 3 / box ** 3)
    ksq_safe = np.where(ksq == 0.0, 1.0, ksq)
    acc = 0.0
    for j, (kj, nj) in enumerate(((k0, n0), (k1, n1), (k2, n2))):
        m = 1j * kj / ksq_safe * amp
        m = np.where(ksq == 0.0, 0.0, m)
        m = np.where(np.abs(nj) == np_side // 2, 0.0, m)
        acc = acc + np.conj(m) * scipy.fft.rfftn(sb[j], workers=FFT_WORKERS)
    return scipy.fft.irfftn(acc, s=(np_side,) * 3, workers=FFT_WORKERS)


# ---------------------------------------------------------------------------
# full reverse pass
# ---------------------------------------------------------------------------
def forward_with_checkpoints(noise, cosmo, box, nm_side, a_grid, geom, shell_chis=None,
                             src_cut=None, interpolation=False, hold=None):
    """Forward model; returns (kappa, states) with states[i] = (x_i, p_i).

    `shell_chis[i]` overrides chi(a_grid[i]) as shell boundary and `src_cut`
    the distances of the in-front-of-source test (to hold the shell partition
    and the source membership fixed while the cosmology varies).
    `interpolation` projects with sub-evolution (project_shell's `sub`);
    `hold` then decides the source membership of moved images at that
    cosmology (project_shell's `hold`)."""
    np_side = noise.shape[0]
    x, p = pm.zeldovich_ic(noise, cosmo, box, nm_side, a_grid[0])
    f = pm.particle_force(x, np_side, nm_side, box)
    states = [(x, p)]
    kappa = np.zeros((len(geom.chi_src), geom.npix, geom.npix))
    for i in range(len(a_grid) - 1):
        x, p, f, p_h = pm.kdk_step(x, p, f, a_grid[i], a_grid[i + 1], cosmo, np_side, nm_side,
                                   box, drift_momentum=True)
        states.append((x, p))
        cb = None if shell_chis is None else (shell_chis[i + 1], shell_chis[i])
        sub = (p_h, 0.5 * (a_grid[i] + a_grid[i + 1])) if interpolation else None
        kappa += lens.project_shell(x, a_grid[i], a_grid[i + 1], cosmo, box, np_side, geom,
                                    chi_bounds=cb, src_cut=src_cut, sub=sub, hold=hold)
    return kappa, states


def kappa_vjp_noise(noise, kappa_bar, cosmo: Cosmology, box, nm_side, a_grid,
                    geom: lens.MapGeometry, interpolation=False):
    """d(sum kappa * kappa_bar)/d noise (Omega_m, sigma_8 fixed), float64.

    Reverse pass over the KDK steps, following the merged force-node
    cotangent f_bar(x_{i+1}) = (K2_i + K1_{i+1}) pbar.  With sub-evolution
    the shell's cotangent of the step's drift momentum p_h = p_{i+1} - K2 f
    joins pbar at the drift (p_h does not pass through f(x_{i+1})).
    """
    np_side = noise.shape[0]
    _, states = forward_with_checkpoints(noise, cosmo, box, nm_side, a_grid, geom,
                                         interpolation=interpolation)
    n = len(a_grid) - 1
    xbar = np.zeros((3, np_side ** 3))
    pbar = np.zeros((3, np_side ** 3))
    fac = []
    for i in range(n):
        a0, a1 = a_grid[i], a_grid[i + 1]
        ah = 0.5 * (a0 + a1)
        fac.append((cosmo.kick_factor(a0, ah, a0), cosmo.drift_factor(a0, a1, ah),
                    cosmo.kick_factor(ah, a1, a1)))
    for i in range(n - 1, -1, -1):
        x1, p1 = states[i + 1]
        k1, dr, k2 = fac[i]
        phbar = 0.0
        if interpolation:
            ph = p1 - k2 * pm.particle_force(x1, np_side, nm_side, box)
            lx, phbar = lens_vjp(x1, a_grid[i], a_grid[i + 1], kappa_bar, cosmo, box, np_side,
                                 geom, sub=(ph, 0.5 * (a_grid[i] + a_grid[i + 1])))
            xbar += lx
        else:
            xbar += lens_vjp(x1, a_grid[i], a_grid[i + 1], kappa_bar, cosmo, box, np_side, geom)
        kf = k2 + (fac[i + 1][0] if i + 1 < n else 0.0)
        xbar += force_vjp(x1, kf * pbar, np_side, nm_side, box)
        pbar = pbar + dr * xbar + phbar
    x0, _ = states[0]
    xbar += force_vjp(x0, fac[0][0] * pbar, np_side, nm_side, box)
    a0 = a_grid[0]
    s_bar = cosmo.D(a0) * xbar + cosmo.gp(a0) * pbar
    return ic_displacement_transpose(s_bar, cosmo, box)


# ---------------------------------------------------------------------------
# cosmology parameters
# ---------------------------------------------------------------------------
def _with_om(cosmo: Cosmology, om):
    return Cosmology(om, cosmo.h, cosmo.n_s, cosmo.sigma8, cosmo.omega_b, cosmo.t_cmb)


def kappa_vjp_cosmo(noise, kappa_bar, cosmo: Cosmology, box, nm_side, a_grid,
                    geom: lens.MapGeometry, dom=1e-5, terms=None, interpolation=False):
    """(noise_bar, d/dOmega_m, d/dsigma_8) of sum(kappa * kappa_bar).

    Omega_m follows the paper's scheme: the reverse pass gives the cotangent
    of every scalar factor (kick K1, drift Dr, kick K2 of each step, the
    growth D(a0) and g_p(a0) of the initial conditions), which is multiplied
    by the central finite difference of that factor in Omega_m; the lens
    projection and the initial displacement field are differenced in
    Omega_m at fixed particle positions / fixed noise.  The shell partition
    (the distance bounds chi(a_i) of the shells, for the particle term and
    the mean term alike) and the test "image in front of source s" are held
    at the central cosmology: membership is piecewise constant and gets no
    gradient.  The lens weight vanishes at chi = chi_s, so holding the source
    membership changes nothing but keeps a difference quotient from
    straddling the kink of (chi_s - chi)_+ when an image lies within
    |dchi_s/dOmega_m| dom of a source plane.  sigma_8 enters only as the
    amplitude of the noise: d/dsigma8 = <noise_bar, noise>/sigma8.
    If `terms` is a list, every additive contribution to d/dOmega_m is
    appended to it (their magnitudes set the conditioning of the sum).
    With `interpolation` the shells use sub-evolution; the drift momentum's
    cotangent joins pbar at the drift, and the shell's Omega_m difference is
    taken at fixed positions and drift momentum, with the source membership
    of each moved image held at its central-cosmology depth.
    """
    np_side = noise.shape[0]
    cp, cm = _with_om(cosmo, cosmo.omega_m + dom), _with_om(cosmo, cosmo.omega_m - dom)
    geom_p = lens.MapGeometry(geom.npix, np.degrees(geom.fov), geom.z_src, cp,
                              rotation_seed=geom.rotation_seed)
    geom_m = lens.MapGeometry(geom.npix, np.degrees(geom.fov), geom.z_src, cm,
                              rotation_seed=geom.rotation_seed)
    _, states = forward_with_checkpoints(noise, cosmo, box, nm_side, a_grid, geom,
                                         interpolation=interpolation)
    n = len(a_grid) - 1

    def factors(c):
        out = []
        for i in range(n):
            a0, a1 = a_grid[i], a_grid[i + 1]
            ah = 0.5 * (a0 + a1)
            out.append(np.array([c.kick_factor(a0, ah, a0), c.drift_factor(a0, a1, ah),
                                 c.kick_factor(ah, a1, a1)]))
        return out
    fac = factors(cosmo)
    dfac = [(p - m) / (2 * dom) for p, m in zip(factors(cp), factors(cm))]
    xbar = np.zeros((3, np_side ** 3))
    pbar = np.zeros((3, np_side ** 3))
    g_om = 0.0

    def add(v):
        if terms is not None:
            terms.append(float(v))
        return float(v)
    for i in range(n - 1, -1, -1):
        x1, p1 = states[i + 1]
        k1, dr, k2 = fac[i]
        f1 = pm.particle_force(x1, np_side, nm_side, box)
        ah = 0.5 * (a_grid[i] + a_grid[i + 1])
        sub = (p1 - k2 * f1, ah) if interpolation else None
        # lens at fixed positions (and drift momenta): cosmology part and
        # position part
        cb = (cosmo.chi(a_grid[i + 1]), cosmo.chi(a_grid[i]))
        kp = lens.project_shell(x1, a_grid[i], a_grid[i + 1], cp, box, np_side, geom_p,
                                chi_bounds=cb, src_cut=geom.chi_src, sub=sub, hold=cosmo)
        km = lens.project_shell(x1, a_grid[i], a_grid[i + 1], cm, box, np_side, geom_m,
                                chi_bounds=cb, src_cut=geom.chi_src, sub=sub, hold=cosmo)
        g_om += add(np.sum(kappa_bar * (kp - km)) / (2 * dom))
        phbar = 0.0
        if interpolation:
            lx, phbar = lens_vjp(x1, a_grid[i], a_grid[i + 1], kappa_bar, cosmo, box, np_side,
                                 geom, sub=sub)
            xbar += lx
        else:
            xbar += lens_vjp(x1, a_grid[i], a_grid[i + 1], kappa_bar, cosmo, box, np_side, geom)
        dot = np.sum(pbar * f1)            # cotangent of K2_i and of K1_{i+1}
        g_om += add(dot * dfac[i][2])
        kf = k2
        if i + 1 < n:
            g_om += add(dot * dfac[i + 1][0])
            kf += fac[i + 1][0]
        xbar += force_vjp(x1, kf * pbar, np_side, nm_side, box)
        ph = p1 - k2 * f1                  # momentum at the half step
        g_om += add(np.sum(xbar * ph) * dfac[i][1])
        pbar = pbar + dr * xbar + phbar
    x0, p0 = states[0]
    f0 = pm.particle_force(x0, np_side, nm_side, box)
    g_om += add(np.sum(pbar * f0) * dfac[0][0])
    xbar += force_vjp(x0, fac[0][0] * pbar, np_side, nm_side, box)
    a0 = a_grid[0]
    s = zeldovich_s = pm.zeldovich_displacement(noise, cosmo, box)
    s_p = pm.zeldovich_displacement(noise, cp, box)
    s_m = pm.zeldovich_displacement(noise, cm, box)
    dD = (cp.D(a0) - cm.D(a0)) / (2 * dom)
    dgp = (cp.gp(a0) - cm.gp(a0)) / (2 * dom)
    ds = (s_p - s_m) / (2 * dom)
    g_om += add(np.sum(xbar * (dD * s + cosmo.D(a0) * ds)))
    g_om += add(np.sum(pbar * (dgp * s + cosmo.gp(a0) * ds)))
    s_bar = cosmo.D(a0) * xbar + cosmo.gp(a0) * pbar
    noise_bar = ic_displacement_transpose(s_bar, cosmo, box)
    g_s8 = float(np.sum(s_bar * zeldovich_s)) / cosmo.sigma8
    return noise_bar, g_om, g_s8
