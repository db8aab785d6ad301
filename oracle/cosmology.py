"""Background cosmology, linear growth and the linear power spectrum (float64).

Test infrastructure only (see the package header).

Follows the paper's appendix on cosmology derivatives: the comoving
distance is c/H0 times the integral of dz / E(z)^(1/2), where the paper's E
is H^2/H0^2 = Om (1+z)^3 + Ok (1+z)^2 + OL, taken flat (Ok = 0,
OL = 1 - Om).  Here `E(a)` denotes H/H0, i.e. the square root of the
paper's E (reading recorded in the design notes).

Linear growth and the kick/drift factors are not printed in the paper; it
states only that FastPM steps particles with kick and drift factors that
reproduce linear displacement exactly in every step (package design
section).  The factors below are derived from that statement:

  momentum   p = a^3 E dx/da
  motion     dx/da = p / (a^3 E),   dp/da = (3/2) Om f / (a^2 E)
  force      f = -grad inv-laplacian(delta)   (what the mesh computes)
  linear     x = q + D s,  f = D s,  p = g_p s,  g_p = a^3 E dD/da
  drift      Dr(a_s, a_e; a_r) = (D(a_e) - D(a_s)) / g_p(a_r)
  kick       K(a_s, a_e; a_r)  = (g_p(a_e) - g_p(a_s)) / D(a_r)

The linear power spectrum is the Eisenstein & Hu (1998) zero-baryon
("no-wiggle") fit, normalised to sigma8 with a real-space top-hat of
8 Mpc/h at a = 1.  The paper uses the EH transfer function for its
cosmology-differentiable variant (appendix); the no-wiggle form is the
requested workload.  Parity of the EH constants is UNPINNED: the paper
prints no P(k) value, so only the transfer function's limits and the sigma8
normalisation are pinned.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate, optimize

C_OVER_H0 = 2997.92458  # c / H0 in Mpc/h


def _quad(f, lo, hi, epsabs=0.0):
    val, _ = integrate.quad(f, lo, hi, epsabs=epsabs, epsrel=1e-13, limit=400)
    return val


class Cosmology:
    """Flat LCDM without radiation, float64 throughout."""

    def __init__(self, omega_m=0.3, h=0.7, n_s=0.96, sigma8=0.8,
                 omega_b=0.05, t_cmb=2.7255):
        self.omega_m = float(omega_m)
        self.h = float(h)
        self.n_s = float(n_s)
        self.sigma8 = float(sigma8)
        self.omega_b = float(omega_b)
        self.t_cmb = float(t_cmb)
        self._du1 = None
        self._amp = None

    # -- background ---------------------------------------------------
    def E(self, a):
        """H(a)/H0 for flat LCDM: sqrt(Om a^-3 + 1 - Om)."""
        a = np.asarray(a, dtype=np.float64)
        return np.sqrt(self.omega_m * a ** -3 + (1.0 - self.omega_m))

    def dE_da(self, a):
        return -1.5 * self.omega_m / (a ** 4 * self.E(a))

    def chi(self, a):
        """Comoving distance to scale factor a, Mpc/h (adaptive quadrature).

        chi(a) = c/H0 * int_a^1 da' / (a'^2 E(a')), the paper's integral over
        z rewritten with dz = -da/a^2.
        """
        f = lambda x: 1.0 / (x * x * math.sqrt(self.omega_m / x ** 3
                                                + 1.0 - self.omega_m))
        if np.ndim(a) == 0:
            return C_OVER_H0 * _quad(f, float(a), 1.0)
        return np.array([C_OVER_H0 * _quad(f, float(v), 1.0)
                         for v in np.ravel(a)]).reshape(np.shape(a))

    def chi_of_z(self, z):
        """c/H0 * int_0^z dz' / E(z') (the paper's form, integrated over z)."""
        f = lambda zz: 1.0 / math.sqrt(self.omega_m * (1 + zz) ** 3
                                       + 1.0 - self.omega_m)
        return C_OVER_H0 * _quad(f, 0.0, float(z))

    # vectorised chi(a) for many scale factors: the same integral after the
    # substitution a' = t^2, which makes the integrand analytic on [0, 1]:
    # chi = 2 c/H0 int_{sqrt a}^1 dt / sqrt(Om + (1 - Om) t^6)
    _GL_X, _GL_W = np.polynomial.legendre.leggauss(32)

    def chi_vec(self, a):
        a = np.asarray(a, dtype=np.float64)
        lo = np.sqrt(a)[..., None]
        half = 0.5 * (1.0 - lo)
        t = lo + half * (self._GL_X + 1.0)
        t2 = t * t
        g = 1.0 / np.sqrt(self.omega_m + (1.0 - self.omega_m) * (t2 * t2 * t2))
        return 2.0 * C_OVER_H0 * np.sum(g * self._GL_W, axis=-1) * half[..., 0]

    def a_of_chi(self, chi):
        """Inverse of chi(a) by Brent's method (scalar)."""
        chi = float(chi)
        if chi <= 0.0:
            return 1.0
        return optimize.brentq(lambda a: self.chi(a) - chi, 1e-4, 1.0,
                               xtol=1e-15, rtol=1e-15, maxiter=200)

    def a_of_chi_vec(self, chi):
        """Inverse of chi(a) for arrays: Newton's method in t = sqrt(a).

        chi(t) = 2 c/H0 int_t^1 g,  d chi/dt = -2 c/H0 g(t),
        g(t) = 1/sqrt(Om + (1 - Om) t^6); chi(t) is nearly linear in t.
        """
        chi = np.asarray(chi, dtype=np.float64)
        t = np.clip(1.0 - chi / (2.0 * C_OVER_H0), 1e-3, 1.0)
        for _ in range(40):
            g = 1.0 / np.sqrt(self.omega_m + (1.0 - self.omega_m) * t ** 6)
            step = (self.chi_vec(t * t) - chi) / (-2.0 * C_OVER_H0 * g)
            t = np.clip(t - step, 1e-4, 1.0)
            if np.all(np.abs(step) <= 1e-15):
                break
        return t * t

    # -- linear growth ------------------------------------------------
    def _growth_integral(self, a):
        """I(a) = int_0^a da' / (a' E(a'))^3."""
        f = lambda x: 1.0 / (x * math.sqrt(self.omega_m / x ** 3
                                           + 1.0 - self.omega_m)) ** 3
        return _quad(f, 0.0, float(a))

    def _du(self, a):
        """Unnormalised growing mode (5 Om / 2) E(a) I(a)."""
        return 2.5 * self.omega_m * float(self.E(a)) * self._growth_integral(a)

    @property
    def du1(self):
        if self._du1 is None:
            self._du1 = self._du(1.0)
        return self._du1

    def D(self, a):
        """Linear growth factor normalised to D(1) = 1."""
        return self._du(a) / self.du1

    # vectorised D(a) for many scale factors: the growth integral after the
    # substitution a' = a u^2, which makes the integrand analytic on [0, 1]:
    # I(a) = 2 a^(5/2) int_0^1 u^4 (Om + (1 - Om) a^3 u^6)^(-3/2) du
    def D_vec(self, a):
        a = np.asarray(a, dtype=np.float64)
        u = 0.5 * (self._GL_X + 1.0)
        a3 = (a ** 3)[..., None]
        g = u ** 4 / (self.omega_m + (1.0 - self.omega_m) * a3 * u ** 6) ** 1.5
        integral = 2.0 * a ** 2.5 * 0.5 * np.sum(g * self._GL_W, axis=-1)
        return 2.5 * self.omega_m * self.E(a) * integral / self.du1

    def dD_da(self, a):
        """dD/da = (5 Om/2) [E'(a) I(a) + 1/(a^3 E^2)] / D_u(1)."""
        a = float(a)
        e = float(self.E(a))
        return 2.5 * self.omega_m * (float(self.dE_da(a)) * self._growth_integral(a)
                                     + 1.0 / (a ** 3 * e * e)) / self.du1

    def dD_da_vec(self, a):
        """Vectorised dD/da: with I(a) = D D_u(1) / ((5 Om / 2) E), the
        derivative of (5 Om / 2) E I / D_u(1) is (E'/E) D + (5 Om / 2) /
        (a^3 E^2 D_u(1))."""
        a = np.asarray(a, dtype=np.float64)
        e = self.E(a)
        return (self.dE_da(a) / e * self.D_vec(a)
                + 2.5 * self.omega_m / (a ** 3 * e * e * self.du1))

    def gp(self, a):
        """g_p(a) = a^3 E(a) dD/da: momentum per unit linear displacement."""
        a = float(a)
        return a ** 3 * float(self.E(a)) * self.dD_da(a)

    def drift_factor(self, a_s, a_e, a_r):
        """Position update per unit momentum at a_r, exact in linear theory."""
        return (self.D(a_e) - self.D(a_s)) / self.gp(a_r)

    def kick_factor(self, a_s, a_e, a_r):
        """Momentum update per unit force at a_r, exact in linear theory."""
        return (self.gp(a_e) - self.gp(a_s)) / self.D(a_r)

    # -- linear power spectrum ----------------------------------------
    def transfer_nowiggle(self, k):
        """Eisenstein & Hu (1998) zero-baryon shape T0(k), k in h/Mpc.

        s      = 44.5 ln(9.83/w_m) / sqrt(1 + 10 w_b^(3/4))      [Mpc]
        alpha  = 1 - 0.328 ln(431 w_m) f_b + 0.38 ln(22.3 w_m) f_b^2
        Gamma  = Om h [alpha + (1 - alpha) / (1 + (0.43 k h s)^4)]
        q      = k Theta^2 / Gamma,  Theta = T_cmb / 2.7
        T0     = L0 / (L0 + C0 q^2),  L0 = ln(2e + 1.8 q),
                 C0 = 14.2 + 731 / (1 + 62.5 q)
        """
        k = np.asarray(k, dtype=np.float64)
        om, h = self.omega_m, self.h
        wm = om * h * h
        wb = self.omega_b * h * h
        fb = self.omega_b / om
        theta = self.t_cmb / 2.7
        s = 44.5 * np.log(9.83 / wm) / np.sqrt(1.0 + 10.0 * wb ** 0.75)
        alpha = 1.0 - 0.328 * np.log(431.0 * wm) * fb \
            + 0.38 * np.log(22.3 * wm) * fb * fb
        gamma = om * h * (alpha + (1.0 - alpha) / (1.0 + (0.43 * k * h * s) ** 4))
        q = k * theta * theta / gamma
        l0 = np.log(2.0 * math.e + 1.8 * q)
        c0 = 14.2 + 731.0 / (1.0 + 62.5 * q)
        return l0 / (l0 + c0 * q * q)

    @staticmethod
    def tophat_window(x):
        """W(x) = 3 (sin x - x cos x) / x^3, series below x = 1e-3."""
        x = np.asarray(x, dtype=np.float64)
        small = np.abs(x) < 1e-3
        xs = np.where(small, 1.0, x)
        w = 3.0 * (np.sin(xs) - xs * np.cos(xs)) / xs ** 3
        return np.where(small, 1.0 - x * x / 10.0, w)

    def _sigma_r_sq_unit(self, r=8.0):
        """sigma_R^2 for unit amplitude A = 1.

        (1 / 2 pi^2) int k^2 k^ns T0^2 W(kR)^2 dk, integrated over ln k up to
        k = 1/R and over k in half-period panels of the window above that,
        truncated at k R = 2400 (the integrand falls as k^-5 there).
        """
        def f_ln(lnk):
            k = math.exp(lnk)
            return k * f_k(k)

        def f_k(k):
            t = float(self.transfer_nowiggle(k))
            w = float(self.tophat_window(k * r))
            return k * k * k ** self.n_s * t * t * w * w / (2.0 * math.pi ** 2)

        total = 0.0
        edges = np.linspace(math.log(1e-7), math.log(1.0 / r), 15)
        for lo, hi in zip(edges[:-1], edges[1:]):
            total += _quad(f_ln, lo, hi, epsabs=1e-24)
        edges = np.arange(1.0 / r, 2400.0 / r, math.pi / r)
        for lo, hi in zip(edges[:-1], edges[1:]):
            total += _quad(f_k, lo, hi, epsabs=1e-24)
        return total

    @property
    def amplitude(self):
        """A such that sigma8 of A k^ns T0^2 equals self.sigma8."""
        if self._amp is None:
            self._amp = self.sigma8 ** 2 / self._sigma_r_sq_unit(8.0)
        return self._amp

    def pk_linear(self, k):
        """Linear matter power at a = 1, (Mpc/h)^3."""
        k = np.asarray(k, dtype=np.float64)
        t = self.transfer_nowiggle(k)
        return self.amplitude * k ** self.n_s * t * t

    def sigma_r(self, r, amplitude=None):
        amp = self.amplitude if amplitude is None else amplitude
        return math.sqrt(amp * self._sigma_r_sq_unit(r))


def lens_prefactor(omega_m):
    """(3/2) Om (H0/c)^2 in (h/Mpc)^2, the prefactor of the convergence
    integral (notation section, Born convergence equation)."""
    return 1.5 * omega_m / C_OVER_H0 ** 2
