"""Born lightcone projection onto convergence maps, float64 (oracle).

Test infrastructure only (see the package header).

The paper's Born convergence (notation section, convergence equation)
is kappa(theta) = (3 H0^2 Om / 2 c^2) int dchi q(chi) delta(chi theta, chi) / a(chi)
with lensing kernel q(chi) = int dchi' n(chi') chi (chi' - chi) / chi'.  For a
source plane n = delta_D(chi' - chi_s) this is q = chi (chi_s - chi) / chi_s.
MADLens evaluates the integral numerically on the lightcone: each PM step
covers a distance shell, the particles of that step are projected, and the
box is replicated where a shell is deeper than the box (package design
section).  Readings fixed here where the paper is silent:

  geometry   flat sky, plane parallel: observer at (L/2, L/2, 0), line of
             sight +axis 2; an image r = x + n L - O has chi = r_2 and
             theta = (r_0 / r_2, r_1 / r_2); the map spans [-T/2, T/2)^2
  shells     step a_i -> a_{i+1} owns chi in (chi(a_{i+1}), chi(a_i)] and
             projects positions at a_{i+1}
  weight     per image w_s = pref V_p (chi_s - chi) / (chi_s chi a(chi) Omega_pix)
             for chi < chi_s, V_p = (L/Np)^3, Omega_pix = dtheta^2, a(chi) per image
  assignment bilinear: t = theta/dtheta + Npix/2 - 1/2, weights to floor(t)
             and floor(t)+1 per axis, contributions off the map dropped
  mean       each shell adds -pref int q(chi)/a(chi) dchi over the shell
             below chi_s to every pixel (the -1 of delta = rho/rho_bar - 1)
  sub-evolution (optional) an image keeps the shell of its end-of-step
             depth and is moved along its step's drift to the scale factor
             of that depth before projection (project_shell's `sub`)

Images are enumerated by brute force over a generous box of replica
offsets; each is tested exactly.  Pins (tests/test_oracle_lens.py): single
particle total and centroid, zero mean for the unperturbed lattice, the
shell partition of a static particle field, linearity in the particle set,
zero signal beyond the source, the 2D paint/gather adjoint identity.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate

from .cosmology import Cosmology, lens_prefactor


class MapGeometry:
    def __init__(self, npix, fov_deg, z_src, cosmo: Cosmology, rotation_seed=None):
        # rotation_seed: None for unrotated replicas, else the seed of the
        # per-replica cube symmetry (replica_symmetry)
        self.rotation_seed = rotation_seed
        self.npix = int(npix)
        self.fov = math.radians(float(fov_deg))
        self.dtheta = self.fov / self.npix
        self.omega_pix = self.dtheta ** 2
        self.z_src = tuple(float(z) for z in z_src)
        self.chi_src = np.array([cosmo.chi_of_z(z) for z in self.z_src])


def bilinear_paint(t0, t1, w, npix):
    """Paint weights w at fractional pixel coordinates (t0, t1) bilinearly."""
    out = np.zeros(npix * npix)
    j0 = np.floor(t0).astype(np.int64)
    j1 = np.floor(t1).astype(np.int64)
    f0 = t0 - j0
    f1 = t1 - j1
    for d0, w0 in ((0, 1.0 - f0), (1, f0)):
        for d1, w1 in ((0, 1.0 - f1), (1, f1)):
            a = j0 + d0
            b = j1 + d1
            ok = (a >= 0) & (a < npix) & (b >= 0) & (b < npix)
            out += np.bincount((a * npix + b)[ok], weights=(w * w0 * w1)[ok],
                               minlength=npix * npix)
    return out.reshape(npix, npix)


def bilinear_gather(t0, t1, kmap):
    """Transpose of bilinear_paint: sum of map values with the same weights."""
    npix = kmap.shape[0]
    out = np.zeros(t0.shape)
    j0 = np.floor(t0).astype(np.int64)
    j1 = np.floor(t1).astype(np.int64)
    f0 = t0 - j0
    f1 = t1 - j1
    for d0, w0 in ((0, 1.0 - f0), (1, f0)):
        for d1, w1 in ((0, 1.0 - f1), (1, f1)):
            a = j0 + d0
            b = j1 + d1
            ok = (a >= 0) & (a < npix) & (b >= 0) & (b < npix)
            v = np.zeros(t0.shape)
            v[ok] = kmap[a[ok], b[ok]]
            out += w0 * w1 * v
    return out


# ---------------------------------------------------------------------------
# replica rotation (the package-design section: the box is rotated before it
# is repeated, to avoid repeated structures along the line of sight)
# ---------------------------------------------------------------------------
_MASK64 = (1 << 64) - 1
# the six axis permutations in lexicographic order; symmetry s of the 48 cube
# symmetries takes permutation s // 8 and flips image axis j when bit j of
# s % 8 is set
PERMS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))


def _mix64(z):
    """The 64-bit finalizer of SplitMix64 (Steele, Lea and Flood, 2014)."""
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
    return z ^ (z >> 31)


def replica_symmetry(nx, ny, nz, seed):
    """Index in [0, 48) of the cube symmetry of replica (nx, ny, nz): the
    offsets are packed as three 21-bit fields (offset by 2^20), mixed, xored
    with the seed, mixed again, reduced modulo 48.  0 is the identity."""
    u = (((nx + (1 << 20)) << 42) | ((ny + (1 << 20)) << 21) | (nz + (1 << 20))) & _MASK64
    return _mix64((int(seed) & _MASK64) ^ _mix64(u)) % 48


def apply_symmetry(v, sym, box=None):
    """Image-frame coordinates of the vectors v ([3][N]) under symmetry sym:
    component j is component perm[j] of v, reflected when flip j is set
    (x -> L - x for positions, given `box`; p -> -p for vectors)."""
    perm = PERMS[sym // 8]
    out = np.empty_like(v)
    for j in range(3):
        c = v[perm[j]]
        if (sym % 8) >> j & 1:
            c = (box - c) if box is not None else -c
        out[j] = c
    return out


def shell_images(x, box, chi_near, chi_far, geom: MapGeometry):
    """All replica images of particles x ([3][N], in [0,L)) in the shell.

    Yields (particle index, r0, r1, chi, sym) arrays for every image with
    chi_near < chi <= chi_far and chi > 0, sym being the replica's cube
    symmetry (0 without rotation); transverse offsets are scanned over a
    range that covers the map plus two pixels at chi_far.  The same chi
    array is yielded for every transverse replica of a depth that shares a
    symmetry.
    """
    half = 0.5 * box
    kxy = int(math.ceil((chi_far * (0.5 * geom.fov + 2 * geom.dtheta) + box) / box)) + 1
    nz_lo = int(math.floor(chi_near / box)) - 1
    nz_hi = int(math.floor(chi_far / box)) + 1
    seed = geom.rotation_seed
    rotated = {}   # symmetry -> positions in the image frame
    for nz in range(nz_lo, nz_hi + 1):
        slabs = {}
        for nx in range(-kxy, kxy + 1):
            for ny in range(-kxy, kxy + 1):
                sym = 0 if seed is None else replica_symmetry(nx, ny, nz, seed)
                if sym not in slabs:
                    if sym not in rotated:
                        rotated[sym] = x if sym == 0 else apply_symmetry(x, sym, box)
                    xr = rotated[sym]
                    rz = xr[2] + nz * box
                    inz = np.nonzero((rz > chi_near) & (rz <= chi_far) & (rz > 0.0))[0]
                    slabs[sym] = (inz, rz[inz], xr)
                inz, chi, xr = slabs[sym]
                if inz.size == 0:
                    continue
                yield inz, xr[0, inz] + nx * box - half, xr[1, inz] + ny * box - half, chi, sym


def project_shell(x, a_far, a_near, cosmo: Cosmology, box, np_side,
                  geom: MapGeometry, include_mean=True, chi_bounds=None, src_cut=None,
                  sub=None, hold: Cosmology = None):
    """Convergence of one PM step's shell, [nsrc][npix][npix].

    x are the positions at a_near (end of the step a_far -> a_near).
    `chi_bounds` = (chi_near, chi_far) overrides the shell's distance range
    (used to hold the shell partition fixed while the cosmology varies).
    `src_cut[s]` overrides chi_s in the test "image in front of source s"
    only (the weight keeps geom.chi_src): it holds that membership fixed
    while the cosmology varies.

    `sub` = (p_h, a_h) turns on sub-evolution (the package-design section's
    sub-evolution step): p_h [3][N] is the momentum the step drifted with and
    a_h its midpoint.  The step's drift moves a particle along
    x(a) = x(a_near) + Dr(a_near, a; a_h) p_h, linear in D(a).  An image keeps
    the shell its end-of-step depth chi_e puts it in, and is moved to
    a_p = a(chi_e), the scale factor of its own distance (one fixed-point
    iteration of chi -> depth of x(a(chi))); its angles, depth, a(chi) and
    weight are then those of the moved image.

    `hold`, with `sub` and `src_cut`: the test "image in front of source s"
    takes the depth the image is moved to under the cosmology `hold` (the
    moved depth changes with the cosmology; holding the test keeps a
    difference quotient in Omega_m from straddling that membership).
    """
    if chi_bounds is None:
        chi_far = float(cosmo.chi(a_far))
        chi_near = float(cosmo.chi(a_near))
    else:
        chi_near, chi_far = (float(v) for v in chi_bounds)
    pref = lens_prefactor(cosmo.omega_m)
    vp = (box / np_side) ** 3
    out = np.zeros((len(geom.chi_src), geom.npix, geom.npix))
    t0s, t1s, chis, chks = [], [], [], []
    # Images that cannot end in front of any source plane carry no weight in
    # any map: they are skipped before their a(chi) (with sub-evolution the
    # slack is the largest move along the step's drift, |Dr| |p_z|).
    cut = [chis_ if src_cut is None else src_cut[s] for s, chis_ in enumerate(geom.chi_src)]
    cmax = max(cut)
    if sub is not None:
        p_h, a_h = sub
        d_near, gp_h = cosmo.D(a_near), cosmo.gp(a_h)
        dr_step = abs(cosmo.drift_factor(a_far, a_near, a_h))
        if hold is not None:
            hd_near, hgp_h = hold.D(a_near), hold.gp(a_h)
    chi_seen = None
    p_rot = {}   # symmetry -> drift momenta in the image frame
    for inz, rx, ry, chi, sym in shell_images(x, box, chi_near, chi_far, geom):
        if chi is not chi_seen:   # the same depth slab for every transverse replica
            chi_seen = chi
            if sub is None:
                sel = np.nonzero(chi < cmax)[0]
                chi_f = chi[sel]
                chi_chk = chi_f
            else:
                if sym not in p_rot:
                    p_rot[sym] = p_h if sym == 0 else apply_symmetry(p_h, sym)
                ph = p_rot[sym]
                sel = np.nonzero(chi - dr_step * np.abs(ph[2, inz]) < cmax)[0]
                isel = inz[sel]
                dr = (cosmo.D_vec(cosmo.a_of_chi_vec(chi[sel])) - d_near) / gp_h
                chi_f = chi[sel] + dr * ph[2, isel]
                chi_chk = chi_f
                if hold is not None:
                    hdr = (hold.D_vec(hold.a_of_chi_vec(chi[sel])) - hd_near) / hgp_h
                    chi_chk = chi[sel] + hdr * ph[2, isel]
        if sel.size == 0:
            continue
        rxs, rys = rx[sel], ry[sel]
        if sub is not None:
            rxs = rxs + dr * ph[0, isel]
            rys = rys + dr * ph[1, isel]
        t0 = rxs / chi_f / geom.dtheta + 0.5 * geom.npix - 0.5
        t1 = rys / chi_f / geom.dtheta + 0.5 * geom.npix - 0.5
        keep = ((t0 > -1.0) & (t0 < geom.npix) & (t1 > -1.0) & (t1 < geom.npix)
                & (chi_f > 0.0))
        t0s.append(t0[keep])
        t1s.append(t1[keep])
        chis.append(chi_f[keep])
        chks.append(chi_chk[keep])
    if chis:
        t0, t1, chi = np.concatenate(t0s), np.concatenate(t1s), np.concatenate(chis)
        chk = np.concatenate(chks)
        a = cosmo.a_of_chi_vec(chi)
        for s, chis_ in enumerate(geom.chi_src):
            src = chk < (chis_ if src_cut is None else src_cut[s])
            if not np.any(src):
                continue
            w = pref * vp * (chis_ - chi[src]) / (chis_ * chi[src] * a[src]
                                                   * geom.omega_pix)
            out[s] += bilinear_paint(t0[src], t1[src], w, geom.npix)
    if include_mean:
        for s, chis in enumerate(geom.chi_src):
            out[s] += shell_mean(cosmo, chi_near, chi_far, chis)
    return out


def shell_mean(cosmo: Cosmology, chi_near, chi_far, chi_s):
    """-pref int_{chi_near}^{min(chi_far, chi_s)} chi (chi_s - chi)/(chi_s a) dchi.

    The integrand is smooth on the shell; 64-point Gauss-Legendre with the
    per-node a(chi) from Newton's method.  (Pinned against adaptive
    quadrature with Brent's root for a(chi) in the tests.)
    """
    hi = min(chi_far, chi_s)
    if hi <= chi_near:
        return 0.0
    pref = lens_prefactor(cosmo.omega_m)
    xg, wg = np.polynomial.legendre.leggauss(64)
    half = 0.5 * (hi - chi_near)
    c = chi_near + half * (xg + 1.0)
    f = c * (chi_s - c) / (chi_s * cosmo.a_of_chi_vec(c))
    return -pref * half * float(np.sum(wg * f))


def shell_mean_adaptive(cosmo: Cosmology, chi_near, chi_far, chi_s):
    """The same integral by adaptive quadrature and Brent's root (slow)."""
    hi = min(chi_far, chi_s)
    if hi <= chi_near:
        return 0.0
    pref = lens_prefactor(cosmo.omega_m)
    f = lambda c: c * (chi_s - c) / (chi_s * cosmo.a_of_chi(c))
    val, _ = integrate.quad(f, chi_near, hi, epsabs=0.0, epsrel=1e-12, limit=200)
    return -pref * val


def run_lensing(noise, cosmo: Cosmology, box, nm_side, a_grid, geom: MapGeometry,
                states=None, interpolation=False, pgd=None):
    """Full forward model: PM run plus the projection after every step.

    Returns (kappa, x_final, p_final).  If `states` is a list, the state
    after each step is appended to it.  `interpolation` projects with
    sub-evolution (project_shell's `sub`).  `pgd` = (alpha0, mu, k_l, k_s)
    projects the positions corrected by the PGD displacement at the step's
    end, alpha = alpha0 a^mu (pm.pgd_displacement), without wrapping them
    back into the box; the run itself goes on from the uncorrected state.
    """
    from . import pm
    np_side = noise.shape[0]
    kappa = np.zeros((len(geom.chi_src), geom.npix, geom.npix))

    def cb(i, x, p, p_h):
        a0, a1 = a_grid[i], a_grid[i + 1]
        sub = (p_h, 0.5 * (a0 + a1)) if interpolation else None
        xp = x
        if pgd is not None:
            # not wrapped back into the box: with rotated replicas, each
            # image moves by its replica's image of the displacement
            alpha0, mu, k_l, k_s = pgd
            xp = x + pm.pgd_displacement(x, np_side, nm_side, box, alpha0 * a1 ** mu, k_l, k_s)
        kappa[...] += project_shell(xp, a0, a1, cosmo, box, np_side, geom, sub=sub)
        if states is not None:
            states.append((x.copy(), p.copy()))

    x, p = pm.run_pm(noise, cosmo, box, nm_side, a_grid, callback=cb,
                     drift_momentum=True)
    return kappa, x, p
