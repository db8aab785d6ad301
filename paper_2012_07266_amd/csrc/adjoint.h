// Host entry points of the reverse-mode kernels (see adjoint.hip).
#pragma once
#include "particles.h"

namespace ml {

// Omega_m dependence of the lens weights at fixed particle position:
// d chi_s / d Omega_m per source and d a(chi) / d Omega_m on the chi grid of
// the a(chi) table (linear interpolation).
// With sub-evolution (LensArgs::sub) also: d D(a(chi)) / d Omega_m on that
// grid, d D(a1) / d Omega_m and d (1 / g_p(a_h)) / d Omega_m of the move, and
// the output array of the drift-momentum cotangent ([3][npart], lattice
// order, Mpc/h, accumulated).
template <class T> struct LensVjpArgs {
    T omega_m;
    T dchis_dom[MAX_SRC];
    const T* dadom;  // [ntab]
    int ntab;
    T dchi;
    const T* ddom = nullptr;  // [ntab]
    T dd_end_dom = T(0);
    T dscale_dom = T(0);
    T* phbar = nullptr;
    __device__ __forceinline__ T dadom_at(T chi) const { return lin_at(dadom, chi); }
    __device__ __forceinline__ T ddom_at(T chi) const { return lin_at(ddom, chi); }
    __device__ __forceinline__ T lin_at(const T* tab, T chi) const {
        T xk = chi / dchi;
        int k = (int)floor(xk);
        k = min(max(k, 0), ntab - 2);
        T s = xk - T(k);
        return (T(1) - s) * tab[k] + s * tab[k + 1];
    }
};

// dots[] slots written by the kernels (double, accumulated):
//   0  sum pbar . f            (cotangent of the kick factors sharing f)
//   1  sum xbar . p_half (mode 0) / sum xbar . s (mode 1)
//   2  sum pbar . s            (mode 1)
//   3  sum sbar . s            (mode 1; sbar written in tile-sorted order)
//   4  lens: sum dw/dOmega_m * gathered kbar
//   5  sum sbar . ds/dOmega_m
//   8.. per-source sums of kbar
template <class T>
void launch_fvjp_readout(Parts<T> p, SortBufs s, Geo g, const T* f0, const T* f1, const T* f2,
                         const T* xbar_in, const T* pbar_in, T H, T ckick, T* xbc, T* fbc,
                         double* dots, uint32_t* fmax_bits, hipStream_t st);
// phbar (may be NULL): a drift-momentum cotangent added to pbar_out in mode 0.
template <class T>
void launch_fvjp_paintgrad(Parts<T> p, SortBufs s, Geo g, const T* rhobar, T mass, const T* xbc,
                           T H, int mode, T dr, T k2, T d0, T gp0, T* xbar_out, const T* pbar_in,
                           T* pbar_out, const T* phbar, T* sb0, T* sb1, T* sb2, double* dots,
                           hipStream_t st);
template <class T>
void launch_dot3(const T* a0, const T* a1, const T* a2, const T* b0, const T* b1, const T* b2,
                 long n, double* dst, hipStream_t st);
template <class T>
void launch_dot_sorted_lattice(Parts<T> p, Geo g, const T* sorted, const T* l0, const T* l1,
                               const T* l2, double* dst, hipStream_t st);
template <class T>
void launch_sorted_to_lattice(Parts<T> p, Geo g, const T* sorted, T* l0, T* l1, T* l2,
                              hipStream_t st);
template <class T>
void launch_map_sums(const T* kbar, int npix, int nsrc, double* dst, hipStream_t st);
template <class T>
void launch_lens_vjp(Parts<T> p, Geo g, const LensArgs<T>& la, const LensVjpArgs<T>& lv,
                     const T* kbar, T* xbar, double* dots, hipStream_t st);

// acc[0] += sum_i c0[i] dots[idx[i]], acc[1] += sum_i c1[i] dots[idx[i]]
// (the cosmology cotangent accumulated on the device, in stream order).
struct CosmoCoef {
    int n = 0;
    int idx[8 + MAX_SRC];
    double c0[8 + MAX_SRC];
    double c1[8 + MAX_SRC];
    void add(int i, double a, double b) {
        idx[n] = i;
        c0[n] = a;
        c1[n] = b;
        ++n;
    }
};
void launch_cosmo_acc(const double* dots, double* acc, const CosmoCoef& c, hipStream_t st);

// ---- forward mode (tangents; tangent arrays [3][npart] in tile order, Mpc/h)
// y = a y + b x over n elements (y not read when a == 0).
template <class T>
void launch_lin(T* y, const T* x, T a, T b, long n, hipStream_t st);
// x_dot = H (D t + cD s), p_dot = H (gp t + cgp s), lattice order; t, s in
// cells; t may alias x_dot.
template <class T>
void launch_ic_tangent(const T* t0, const T* t1, const T* t2, const T* s0, const T* s1,
                       const T* s2, T* xd, T* pd, T D, T gp, T cD, T cgp, T H, long n,
                       hipStream_t st);
// sorted[a][k] = lattice[a][L(k)] for the current tile order.
template <class T>
void launch_lattice_to_sorted(Parts<T> p, Geo g, const T* lat, T* sorted, hipStream_t st);
// Tangent of a step's first half-kick and drift at the state before it.
template <class T>
void launch_jvp_pre(Parts<T> p, Geo g, T* xdot, T* pdot, const T* fdot, T H, T k1, T dr, T ck1,
                    T cdr, hipStream_t st);
// Readout part of the force tangent on the force meshes f0..f2 into fbc
// (cells), and a bound for the tangent paint's scale to vmax_bits.
template <class T>
void launch_fjvp_gather(Parts<T> p, SortBufs s, Geo g, const T* f0, const T* f1, const T* f2,
                        const T* xdot, T invH, T mass, T* fbc, uint32_t* vmax_bits,
                        hipStream_t st);
// Paint part of the force tangent from the tangent force meshes m0..m2, the
// second half-kick of p_dot (pdot may be NULL) and f_dot.
template <class T>
void launch_fjvp_readout_kick(Parts<T> p, SortBufs s, Geo g, const T* m0, const T* m1, const T* m2,
                              const T* fbc, T H, T k2, T ck2, T* pdot, T* fdot, hipStream_t st);
// Lens projection tangent (particle term, plus om_dot times the weights'
// Omega_m derivative) accumulated into kdot [nsrc][npix][npix].  With
// sub-evolution (la.sub) the drift momentum's tangent is pdot - K2 fdot -
// ck2 f (ck2 = om_dot dK2/dOm).
template <class T>
void launch_lens_jvp(Parts<T> p, Geo g, const LensArgs<T>& la, const LensVjpArgs<T>& lv,
                     const T* xdot, const T* pdot, const T* fdot, T ck2, T om_dot, T* kdot,
                     hipStream_t st);
// kdot[s] += mv.v[s] on every pixel.
template <class T>
void launch_map_add(T* kdot, int npix, int nsrc, const MapAdd<T>& mv, hipStream_t st);

}  // namespace ml
