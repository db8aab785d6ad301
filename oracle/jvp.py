"""Jacobian-vector products (forward-mode tangents) of the forward model,
float64 (oracle).

Test infrastructure only (see the package header).

The paper's automatic differentiation provides both directional derivatives
(Jvp) and gradients (vJp) of the convergence maps; every derivative check
it shows (one perturbed initial-condition pixel, sigma_8, Omega_m with
single-mode initial conditions) is a Jvp against a finite difference
(section on validating the derivatives).  Its cosmology dependence goes
through finite differences of the scalar factors (appendix on cosmology
derivatives).  This module writes the tangent pass out by hand, for a
direction (noise_dot, Om_dot, s8_dot):

  initial   s = S(noise; Om, s8), x0 = q + D s, p0 = g_p s
            s_dot = S(noise_dot) + (s8_dot / s8) s + Om_dot dS/dOm
            x0_dot = D s_dot + Om_dot (dD/dOm) s,  p0_dot = g_p s_dot + Om_dot (dg_p/dOm) s
  force     f = R(x, M(P(x))):
            f_dot_j = x_dot . grad R(x, M_j)  +  R(x, M_j(P'(x) x_dot))
            with the tangent paint P'(x) x_dot = mass sum_p sum_a dW/du_a xdot_a / H
  KDK step  ph = p + K1 f;             ph_dot = p_dot + K1 f_dot + Om_dot K1' f
            x' = x + Dr ph;            x'_dot = x_dot + Dr ph_dot + Om_dot Dr' ph
            p' = ph + K2 f(x');        p'_dot = ph_dot + K2 f'_dot + Om_dot K2' f'
  lens      per image: kappa += w(chi) B(t), t = (r_perp / chi) / dtheta + c;
            kappa_dot += (dw/dchi chi_dot) B + w (dB/dt . t_dot),
            t_dot = (r_perp_dot - r_perp chi_dot / chi) / (chi dtheta);
            plus Om_dot times the central difference of the shell in Om at
            fixed positions, shell partition and source membership
  K1', Dr', K2', dD/dOm, dg_p/dOm and dS/dOm are central differences in Om
  of the same step size as the reverse pass (adjoint.kappa_vjp_cosmo).

The CIC and bilinear derivatives are one-sided at integer coordinates,
consistent with floor (the same convention as the adjoint).  Pins
(tests/test_oracle_jvp.py): central finite differences of the forward
oracle for the tangent paint, the force, the lens, one perturbed noise pixel
of the whole model, sigma_8 and Omega_m; the transpose identity
<kbar, J v> = <J^T kbar, v> against the reverse pass; linearity.
"""
from __future__ import annotations

import numpy as np
import scipy.fft

from . import lens, pm
from .adjoint import cic_gradient_gather, forward_with_checkpoints
from .cosmology import Cosmology, lens_prefactor

FFT_WORKERS = -1


# ---------------------------------------------------------------------------
# force node
# ---------------------------------------------------------------------------
def cic_paint_tangent(x, x_dot, nm_side, box, mass):
    """d/de of cic_paint(x + e x_dot, mass): [Nm]^3.

    Corner c of particle p receives mass sum_a (dW_c/du_a) x_dot_a / H with
    W_c = prod_a w_a, w_a = 1 - t_a or t_a, dw_a/du_a = -1 or +1.
    """
    h = box / nm_side
    i, t = pm.cic_weights(x, nm_side, box)
    out = np.zeros(nm_side ** 3)
    u_dot = x_dot / h
    for c0 in (0, 1):
        for c1 in (0, 1):
            for c2 in (0, 1):
                c = (c0, c1, c2)
                idx = [(i[d] + c[d]) % nm_side for d in range(3)]
                flat = (idx[0] * nm_side + idx[1]) * nm_side + idx[2]
                w = [t[d] if c[d] else 1.0 - t[d] for d in range(3)]
                dw = [1.0 if c[d] else -1.0 for d in range(3)]
                val = (dw[0] * w[1] * w[2] * u_dot[0] + w[0] * dw[1] * w[2] * u_dot[1]
                       + w[0] * w[1] * dw[2] * u_dot[2])
                out += np.bincount(flat, weights=mass * val, minlength=nm_side ** 3)
    return out.reshape((nm_side,) * 3)


def force_operator(mesh, box):
    """The linear Fourier force operator M: irfftn(i k_j / k^2 rfftn(mesh)),
    zero at k = 0 and on the plane |n_j| = N/2 (pm.force_mesh without the
    mean subtraction, which a tangent does not carry)."""
    n = mesh.shape[0]
    comps = pm.gradient_inverse_laplacian(scipy.fft.rfftn(mesh, workers=FFT_WORKERS), n, box)
    return np.stack([scipy.fft.irfftn(c, s=(n,) * 3, workers=FFT_WORKERS) for c in comps])


def force_jvp(x, x_dot, np_side, nm_side, box):
    """Tangent of f(x) = particle_force(x) along x_dot: [3][N] (Mpc/h)."""
    mass = (nm_side / np_side) ** 3
    fmesh = pm.force_mesh(pm.density(x, np_side, nm_side, box), box)
    f_dot = np.zeros_like(x)
    for j in range(3):   # readout part: the force meshes' gradient along x_dot
        f_dot[j] = np.sum(x_dot * cic_gradient_gather(x, fmesh[j], box), axis=0)
    m_dot = force_operator(cic_paint_tangent(x, x_dot, nm_side, box, mass), box)
    for j in range(3):   # paint part: the force of the density tangent
        f_dot[j] += pm.cic_readout(x, m_dot[j], box)
    return f_dot


# ---------------------------------------------------------------------------
# lens projection
# ---------------------------------------------------------------------------
def bilinear_paint_tangent(t0, t1, c, c0, c1, npix):
    """Paint c B + c0 dB/dt0 + c1 dB/dt1 per point, B the bilinear weights of
    lens.bilinear_paint (corners off the map dropped)."""
    out = np.zeros(npix * npix)
    j0 = np.floor(t0).astype(np.int64)
    j1 = np.floor(t1).astype(np.int64)
    f0 = t0 - j0
    f1 = t1 - j1
    for d0, w0, dw0 in ((0, 1.0 - f0, -1.0), (1, f0, 1.0)):
        for d1, w1, dw1 in ((0, 1.0 - f1, -1.0), (1, f1, 1.0)):
            a = j0 + d0
            b = j1 + d1
            ok = (a >= 0) & (a < npix) & (b >= 0) & (b < npix)
            v = c * w0 * w1 + c0 * dw0 * w1 + c1 * w0 * dw1
            out += np.bincount((a * npix + b)[ok], weights=v[ok], minlength=npix * npix)
    return out.reshape(npix, npix)


def lens_jvp(x, x_dot, a_far, a_near, cosmo: Cosmology, box, np_side, geom: lens.MapGeometry,
             sub=None, ph_dot=None):
    """Tangent of the shell's convergence (particle term) along x_dot at
    fixed cosmology: [nsrc][npix][npix].

    With `sub` = (p_h, a_h) (sub-evolution) the image at end-of-step depth
    chi_e is projected at r' = r + dr(chi_e) p_h, whose tangent is
    r'_dot = r_dot + (d dr / d chi_e) r_dot_z p_h + dr p_h_dot (p_h_dot the
    drift momentum's tangent, zero if None); the splat's tangent is then
    taken at r' along r'_dot."""
    chi_far = float(cosmo.chi(a_far))
    chi_near = float(cosmo.chi(a_near))
    pref = lens_prefactor(cosmo.omega_m)
    vp = (box / np_side) ** 3
    out = np.zeros((len(geom.chi_src), geom.npix, geom.npix))
    c = 0.5 * geom.npix - 0.5
    if sub is not None:
        p_h, a_h = sub
        d_near, gp_h = cosmo.D(a_near), cosmo.gp(a_h)
        if ph_dot is None:
            ph_dot = np.zeros_like(p_h)
    for idx, rx, ry, chi, sym in lens.shell_images(x, box, chi_near, chi_far, geom):
        # tangent in the image frame: image axis j is box axis perm[j],
        # reflected when flip j is set
        perm, flips = lens.PERMS[sym // 8], sym % 8
        sgn = [-1.0 if flips >> j & 1 else 1.0 for j in range(3)]
        xd = [sgn[j] * x_dot[perm[j], idx] for j in range(3)]
        if sub is not None:
            q = [sgn[j] * p_h[perm[j], idx] for j in range(3)]
            qd = [sgn[j] * ph_dot[perm[j], idx] for j in range(3)]
            ae = cosmo.a_of_chi_vec(chi)
            dr = (cosmo.D_vec(ae) - d_near) / gp_h
            ddr = cosmo.dD_da_vec(ae) * (-ae * ae * cosmo.E(ae) / 2997.92458) / gp_h
            zd = xd[2]
            xd = [xd[j] + ddr * zd * q[j] + dr * qd[j] for j in range(3)]
            rx = rx + dr * q[0]
            ry = ry + dr * q[1]
            chi = chi + dr * q[2]
        t0 = rx / chi / geom.dtheta + c
        t1 = ry / chi / geom.dtheta + c
        keep = (t0 > -1.0) & (t0 < geom.npix) & (t1 > -1.0) & (t1 < geom.npix) & (chi > 0.0)
        if not np.any(keep):
            continue
        idx, rx, ry, chi, t0, t1 = idx[keep], rx[keep], ry[keep], chi[keep], t0[keep], t1[keep]
        xd = [v[keep] for v in xd]
        a = cosmo.a_of_chi_vec(chi)
        dadchi = -a * a * cosmo.E(a) / 2997.92458
        for s, chis in enumerate(geom.chi_src):
            src = chi < chis
            if not np.any(src):
                continue
            ch, aa, da = chi[src], a[src], dadchi[src]
            g = (chis - ch) / (chis * ch * aa)
            w = pref * vp * g / geom.omega_pix
            dg = -1.0 / (chis * ch * aa) - g / ch - g * da / aa
            dw = pref * vp * dg / geom.omega_pix
            zd = xd[2][src]
            inv = 1.0 / (ch * geom.dtheta)
            td0 = (xd[0][src] - rx[src] * zd / ch) * inv
            td1 = (xd[1][src] - ry[src] * zd / ch) * inv
            out[s] += bilinear_paint_tangent(t0[src], t1[src], dw * zd, w * td0, w * td1,
                                             geom.npix)
    return out


def _with_om(cosmo: Cosmology, om):
    return Cosmology(om, cosmo.h, cosmo.n_s, cosmo.sigma8, cosmo.omega_b, cosmo.t_cmb)


def _geom_at(geom: lens.MapGeometry, cosmo: Cosmology):
    return lens.MapGeometry(geom.npix, np.degrees(geom.fov), geom.z_src, cosmo,
                            rotation_seed=geom.rotation_seed)


def lens_om_tangent(x, a_far, a_near, cosmo: Cosmology, box, np_side, geom: lens.MapGeometry,
                    dom=1e-5, sub=None):
    """d kappa_shell / d Omega_m at fixed positions (and drift momenta, with
    `sub`): central difference with the shell's distance bounds and the
    source membership held at the central cosmology (membership is piecewise
    constant), mean term included."""
    cp, cm = _with_om(cosmo, cosmo.omega_m + dom), _with_om(cosmo, cosmo.omega_m - dom)
    cb = (cosmo.chi(a_near), cosmo.chi(a_far))
    kp = lens.project_shell(x, a_far, a_near, cp, box, np_side, _geom_at(geom, cp),
                            chi_bounds=cb, src_cut=geom.chi_src, sub=sub, hold=cosmo)
    km = lens.project_shell(x, a_far, a_near, cm, box, np_side, _geom_at(geom, cm),
                            chi_bounds=cb, src_cut=geom.chi_src, sub=sub, hold=cosmo)
    return (kp - km) / (2 * dom)


# ---------------------------------------------------------------------------
# initial conditions and the KDK step
# ---------------------------------------------------------------------------
def ic_jvp(noise, noise_dot, om_dot, s8_dot, cosmo: Cosmology, box, a0, dom=1e-5):
    """(x0_dot, p0_dot) of the Zel'dovich initial conditions: [3][N] each."""
    s = pm.zeldovich_displacement(noise, cosmo, box)
    s_dot = pm.zeldovich_displacement(noise_dot, cosmo, box) + (s8_dot / cosmo.sigma8) * s
    cp, cm = _with_om(cosmo, cosmo.omega_m + dom), _with_om(cosmo, cosmo.omega_m - dom)
    if om_dot != 0.0:
        ds = (pm.zeldovich_displacement(noise, cp, box)
              - pm.zeldovich_displacement(noise, cm, box)) / (2 * dom)
        s_dot = s_dot + om_dot * ds
    d_dom = (cp.D(a0) - cm.D(a0)) / (2 * dom)
    gp_dom = (cp.gp(a0) - cm.gp(a0)) / (2 * dom)
    x_dot = cosmo.D(a0) * s_dot + om_dot * d_dom * s
    p_dot = cosmo.gp(a0) * s_dot + om_dot * gp_dom * s
    return x_dot, p_dot


def step_factors(cosmo: Cosmology, a0, a1):
    """(K1, Dr, K2) of the KDK step a0 -> a1."""
    ah = 0.5 * (a0 + a1)
    return np.array([cosmo.kick_factor(a0, ah, a0), cosmo.drift_factor(a0, a1, ah),
                     cosmo.kick_factor(ah, a1, a1)])


def step_jvp(x, p, f, x_dot, p_dot, f_dot, a0, a1, om_dot, cosmo: Cosmology, np_side,
             nm_side, box, dom=1e-5):
    """One KDK step and its tangent.  Returns (x, p, f, x_dot, p_dot, f_dot)
    at a1; f, f_dot are the force and its tangent at the new positions."""
    k1, dr, k2 = step_factors(cosmo, a0, a1)
    dk1, ddr, dk2 = (step_factors(_with_om(cosmo, cosmo.omega_m + dom), a0, a1)
                     - step_factors(_with_om(cosmo, cosmo.omega_m - dom), a0, a1)) / (2 * dom)
    ph = p + k1 * f
    ph_dot = p_dot + k1 * f_dot + om_dot * dk1 * f
    x1 = np.mod(x + dr * ph, box)
    x1_dot = x_dot + dr * ph_dot + om_dot * ddr * ph
    f1 = pm.particle_force(x1, np_side, nm_side, box)
    f1_dot = force_jvp(x1, x1_dot, np_side, nm_side, box)
    p1 = ph + k2 * f1
    p1_dot = ph_dot + k2 * f1_dot + om_dot * dk2 * f1
    return x1, p1, f1, x1_dot, p1_dot, f1_dot


# ---------------------------------------------------------------------------
# whole model
# ---------------------------------------------------------------------------
def kappa_jvp(noise, noise_dot, om_dot, s8_dot, cosmo: Cosmology, box, nm_side, a_grid,
              geom: lens.MapGeometry, dom=1e-5, interpolation=False):
    """(kappa, kappa_dot): the maps and their directional derivative along
    (noise_dot, Om_dot, s8_dot).  `interpolation` projects with
    sub-evolution; the drift momentum p_h = p - K2 f and its tangent
    p_dot - K2 f_dot - Om_dot K2' f enter the shell's tangent."""
    np_side = noise.shape[0]
    x, p = pm.zeldovich_ic(noise, cosmo, box, nm_side, a_grid[0])
    x_dot, p_dot = ic_jvp(noise, noise_dot, om_dot, s8_dot, cosmo, box, a_grid[0], dom)
    f = pm.particle_force(x, np_side, nm_side, box)
    f_dot = force_jvp(x, x_dot, np_side, nm_side, box)
    shape = (len(geom.chi_src), geom.npix, geom.npix)
    kappa, kappa_dot = np.zeros(shape), np.zeros(shape)
    for i in range(len(a_grid) - 1):
        a0, a1 = a_grid[i], a_grid[i + 1]
        x, p, f, x_dot, p_dot, f_dot = step_jvp(x, p, f, x_dot, p_dot, f_dot, a0, a1, om_dot,
                                                cosmo, np_side, nm_side, box, dom)
        sub, ph_dot = None, None
        if interpolation:
            k2 = step_factors(cosmo, a0, a1)[2]
            dk2 = (step_factors(_with_om(cosmo, cosmo.omega_m + dom), a0, a1)[2]
                   - step_factors(_with_om(cosmo, cosmo.omega_m - dom), a0, a1)[2]) / (2 * dom)
            sub = (p - k2 * f, 0.5 * (a0 + a1))
            ph_dot = p_dot - k2 * f_dot - om_dot * dk2 * f
        kappa += lens.project_shell(x, a0, a1, cosmo, box, np_side, geom, sub=sub)
        kappa_dot += lens_jvp(x, x_dot, a0, a1, cosmo, box, np_side, geom, sub=sub, ph_dot=ph_dot)
        if om_dot != 0.0:
            kappa_dot += om_dot * lens_om_tangent(x, a0, a1, cosmo, box, np_side, geom, dom,
                                                  sub=sub)
    return kappa, kappa_dot


def kappa_at(noise, cosmo: Cosmology, box, nm_side, a_grid, geom: lens.MapGeometry,
             shell_chis=None, src_cut=None):
    """The forward maps, optionally with the shell partition and source
    membership held (for finite differences in Omega_m)."""
    k, _ = forward_with_checkpoints(noise, cosmo, box, nm_side, a_grid, geom,
                                    shell_chis=shell_chis, src_cut=src_cut)
    return k
