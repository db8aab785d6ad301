// Float64 host background for the device kernels: flat LCDM expansion,
// comoving distance and its inverse, linear growth, FastPM-type kick and
// drift factors, Eisenstein-Hu no-wiggle linear power normalised to sigma8,
// and the lensing kernel's per-shell mean term.
//
// The comoving distance is c/H0 times the integral of dz over the square
// root of the paper's E(z) = Om (1+z)^3 + OL with OL = 1 - Om (appendix on
// cosmology derivatives).  Growth and the kick/drift factors follow from the
// design section's statement that every step reproduces linear displacement
// exactly: with p = a^3 H/H0 dx/da, a linear displacement x = q + D s has
// p = g_p s with g_p = a^3 (H/H0) dD/da and force f = D s, so
//   drift  Dr(a_s, a_e; a_r) = (D(a_e) - D(a_s)) / g_p(a_r)
//   kick   K(a_s, a_e; a_r)  = (g_p(a_e) - g_p(a_s)) / D(a_r).
#pragma once

namespace ml {

constexpr double C_H0 = 2997.92458;  // c/H0 in Mpc/h

struct HostCosmo {
    double om = 0.3, h = 0.7, ns = 0.96, s8 = 0.8, ob = 0.05, tcmb = 2.7255;
    double du1 = 1.0;  // unnormalised growth at a = 1
    double amp = 1.0;  // P(k) amplitude giving sigma8

    void init(double omega_m, double hh, double n_s, double sigma8, double omega_b,
              double t_cmb);
    double E(double a) const;               // H/H0
    double chi(double a) const;             // Mpc/h
    double chi_of_z(double z) const { return chi(1.0 / (1.0 + z)); }
    double a_of_chi(double c) const;
    // a(k dchi) for k = 0..n-1, marching outward from a = 1 (same accuracy as
    // a_of_chi, far fewer distance integrals)
    void a_of_chi_grid(double dchi, int n, double* a_out) const;
    double dadchi(double a) const;          // da/dchi = -a^2 E / (c/H0)
    // D(a_k) and dD/da(a_k) for a monotonic grid a_k (one growth integral
    // at the smallest a, then one Gauss-Legendre panel per interval upward)
    void growth_grid(const double* a, int n, double* d_out, double* dda_out) const;
    double D(double a) const;
    double dDda(double a) const;
    double gp(double a) const;
    double drift(double as, double ae, double ar) const { return (D(ae) - D(as)) / gp(ar); }
    double kick(double as, double ae, double ar) const { return (gp(ae) - gp(as)) / D(ar); }
    double transfer(double k) const;        // EH98 zero-baryon T0(k), k in h/Mpc
    double pk(double k) const;              // linear P(k) at a = 1, (Mpc/h)^3
    // -(3/2) Om (H0/c)^2 int_{lo}^{min(hi, cs)} chi (cs - chi) / (cs a(chi)) dchi
    double shell_mean(double lo, double hi, double cs) const;

  private:
    double growth_integral(double a) const;
    double du(double a) const;
};

}  // namespace ml
