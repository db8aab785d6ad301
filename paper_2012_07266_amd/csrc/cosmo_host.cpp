// Float64 host background (see cosmo_host.h).  All integrals use composite
// Gauss-Legendre quadrature after substitutions that make the integrands
// smooth: a = t^2 turns the distance integrand into 1/sqrt(Om + (1-Om) t^6)
// and the growth integrand into 2 t^4 / (Om + (1-Om) t^6)^(3/2).
#include "cosmo_host.h"

#include <cmath>

namespace ml {

namespace {

constexpr int GLN = 16;

struct GL16 {
    double x[GLN], w[GLN];
    GL16() {
        // nodes of the Legendre polynomial P_16 by Newton's method from the
        // Chebyshev-like start cos(pi (i + 3/4) / (n + 1/2))
        const double pi = 3.14159265358979323846;
        for (int i = 0; i < GLN; ++i) {
            double z = std::cos(pi * (i + 0.75) / (GLN + 0.5));
            double dp = 1.0;
            for (int it = 0; it < 100; ++it) {
                double p0 = 1.0, p1 = 0.0;
                for (int j = 1; j <= GLN; ++j) {
                    double p2 = p1;
                    p1 = p0;
                    p0 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p2) / j;
                }
                dp = GLN * (z * p0 - p1) / (z * z - 1.0);
                double dz = p0 / dp;
                z -= dz;
                if (std::fabs(dz) < 1e-16) break;
            }
            x[i] = z;
            w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
        }
    }
};

const GL16& gl() {
    static GL16 g;
    return g;
}

template <class F> double integrate(F f, double lo, double hi, int panels) {
    const GL16& g = gl();
    double total = 0.0, step = (hi - lo) / panels;
    for (int p = 0; p < panels; ++p) {
        double a = lo + p * step, half = 0.5 * step, mid = a + half;
        double s = 0.0;
        for (int i = 0; i < GLN; ++i) s += g.w[i] * f(mid + half * g.x[i]);
        total += s * half;
    }
    return total;
}

double tophat(double x) {
    if (std::fabs(x) < 1e-3) return 1.0 - x * x / 10.0;
    return 3.0 * (std::sin(x) - x * std::cos(x)) / (x * x * x);
}

}  // namespace

void HostCosmo::init(double omega_m, double hh, double n_s, double sigma8, double omega_b,
                     double t_cmb) {
    om = omega_m;
    h = hh;
    ns = n_s;
    s8 = sigma8;
    ob = omega_b;
    tcmb = t_cmb;
    du1 = du(1.0);
    // sigma8 normalisation: (1/2pi^2) int k^3 P W(8k)^2 dlnk
    const double R = 8.0, pi = 3.14159265358979323846;
    auto f_ln = [&](double lnk) {
        double k = std::exp(lnk), t = transfer(k), w = tophat(k * R);
        return k * k * k * std::pow(k, ns) * t * t * w * w;
    };
    auto f_k = [&](double k) {
        double t = transfer(k), w = tophat(k * R);
        return k * k * std::pow(k, ns) * t * t * w * w;
    };
    double s = integrate(f_ln, std::log(1e-7), std::log(1.0 / R), 64);
    double klo = 1.0 / R;
    const double kstep = pi / R;
    while (klo < 2400.0 / R) {
        s += integrate(f_k, klo, klo + kstep, 1);
        klo += kstep;
    }
    s /= 2.0 * pi * pi;
    amp = s8 * s8 / s;
}

double HostCosmo::E(double a) const { return std::sqrt(om / (a * a * a) + 1.0 - om); }

double HostCosmo::chi(double a) const {
    if (a >= 1.0) return 0.0;
    auto g = [&](double t) {
        double t2 = t * t;
        return 1.0 / std::sqrt(om + (1.0 - om) * t2 * t2 * t2);
    };
    return 2.0 * C_H0 * integrate(g, std::sqrt(a), 1.0, 4);
}

double HostCosmo::a_of_chi(double c) const {
    if (c <= 0.0) return 1.0;
    // Newton in t = sqrt(a): d chi / dt = -2 (c/H0) / sqrt(Om + (1-Om) t^6)
    double t = 1.0 - c / (2.0 * C_H0);
    if (t < 1e-3) t = 1e-3;
    for (int it = 0; it < 60; ++it) {
        double t2 = t * t;
        double g = 1.0 / std::sqrt(om + (1.0 - om) * t2 * t2 * t2);
        double step = (chi(t2) - c) / (-2.0 * C_H0 * g);
        t -= step;
        if (t < 1e-4) t = 1e-4;
        if (t > 1.0) t = 1.0;
        if (std::fabs(step) < 1e-15) break;
    }
    return t * t;
}

void HostCosmo::a_of_chi_grid(double dchi, int n, double* a_out) const {
    // chi(t) = 2 (c/H0) int_t^1 g, g(t) = 1/sqrt(Om + (1-Om) t^6), t = sqrt(a).
    // Node k starts Newton's method from node k-1 and measures chi(t) as
    // chi(t_prev) plus the integral over [t, t_prev] (one Gauss-Legendre
    // panel on an interval of one table step).
    auto g = [&](double t) {
        double t2 = t * t;
        return 1.0 / std::sqrt(om + (1.0 - om) * t2 * t2 * t2);
    };
    if (n <= 0) return;
    a_out[0] = 1.0;
    double t_prev = 1.0, chi_prev = 0.0;
    for (int k = 1; k < n; ++k) {
        const double c = k * dchi;
        double t = t_prev - (c - chi_prev) / (2.0 * C_H0 * g(t_prev));
        if (t < 1e-4) t = 1e-4;
        double chi_t = chi_prev;
        for (int it = 0; it < 50; ++it) {
            chi_t = chi_prev + 2.0 * C_H0 * integrate(g, t, t_prev, 1);
            double step = (chi_t - c) / (-2.0 * C_H0 * g(t));
            t -= step;
            if (t < 1e-4) t = 1e-4;
            if (std::fabs(step) < 1e-15) break;
        }
        chi_prev = chi_prev + 2.0 * C_H0 * integrate(g, t, t_prev, 1);
        t_prev = t;
        a_out[k] = t * t;
    }
}

double HostCosmo::dadchi(double a) const { return -a * a * E(a) / C_H0; }

double HostCosmo::growth_integral(double a) const {
    auto f = [&](double t) {
        double t2 = t * t;
        double q = om + (1.0 - om) * t2 * t2 * t2;
        return 2.0 * t2 * t2 / (q * std::sqrt(q));
    };
    return integrate(f, 0.0, std::sqrt(a), 4);
}

double HostCosmo::du(double a) const { return 2.5 * om * E(a) * growth_integral(a); }

void HostCosmo::growth_grid(const double* a, int n, double* d_out, double* dda_out) const {
    if (n <= 0) return;
    // integrand of growth_integral in t = sqrt(a)
    auto f = [&](double t) {
        double t2 = t * t;
        double q = om + (1.0 - om) * t2 * t2 * t2;
        return 2.0 * t2 * t2 / (q * std::sqrt(q));
    };
    const bool up = a[n - 1] >= a[0];  // index order of increasing a
    int k = up ? 0 : n - 1;
    const int dk = up ? 1 : -1;
    double t_prev = std::sqrt(a[k]);
    double integral = growth_integral(a[k]);
    for (int i = 0; i < n; ++i, k += dk) {
        const double t = std::sqrt(a[k]);
        if (i > 0) integral += integrate(f, t_prev, t, 1);
        t_prev = t;
        const double e = E(a[k]);
        d_out[k] = 2.5 * om * e * integral / du1;
        const double de = -1.5 * om / (a[k] * a[k] * a[k] * a[k] * e);
        dda_out[k] = 2.5 * om * (de * integral + 1.0 / (a[k] * a[k] * a[k] * e * e)) / du1;
    }
}

double HostCosmo::D(double a) const { return du(a) / du1; }

double HostCosmo::dDda(double a) const {
    double e = E(a);
    double de = -1.5 * om / (a * a * a * a * e);
    return 2.5 * om * (de * growth_integral(a) + 1.0 / (a * a * a * e * e)) / du1;
}

double HostCosmo::gp(double a) const { return a * a * a * E(a) * dDda(a); }

double HostCosmo::transfer(double k) const {
    double wm = om * h * h, wb = ob * h * h, fb = ob / om;
    double theta = tcmb / 2.7;
    double s = 44.5 * std::log(9.83 / wm) / std::sqrt(1.0 + 10.0 * std::pow(wb, 0.75));
    double alpha = 1.0 - 0.328 * std::log(431.0 * wm) * fb + 0.38 * std::log(22.3 * wm) * fb * fb;
    double ks = 0.43 * k * h * s;
    double gamma = om * h * (alpha + (1.0 - alpha) / (1.0 + ks * ks * ks * ks));
    double q = k * theta * theta / gamma;
    double l0 = std::log(2.0 * 2.71828182845904523536 + 1.8 * q);
    double c0 = 14.2 + 731.0 / (1.0 + 62.5 * q);
    return l0 / (l0 + c0 * q * q);
}

double HostCosmo::pk(double k) const {
    double t = transfer(k);
    return amp * std::pow(k, ns) * t * t;
}

double HostCosmo::shell_mean(double lo, double hi, double cs) const {
    double top = hi < cs ? hi : cs;
    if (top <= lo) return 0.0;
    auto f = [&](double c) { return c * (cs - c) / (cs * a_of_chi(c)); };
    double pref = 1.5 * om / (C_H0 * C_H0);
    return -pref * integrate(f, lo, top, 4);
}

}  // namespace ml
