// Host entry points of the reverse-mode kernels (see adjoint.hip).
#pragma once
#include "particles.h"

namespace ml {

// Omega_m dependence of the lens weights at fixed particle position:
// d chi_s / d Omega_m per source and d a(chi) / d Omega_m on the chi grid of
// the a(chi) table (linear interpolation).
template <class T> struct LensVjpArgs {
    T omega_m;
    T dchis_dom[MAX_SRC];
    const T* dadom;  // [ntab]
    int ntab;
    T dchi;
    __device__ __forceinline__ T dadom_at(T chi) const {
        T xk = chi / dchi;
        int k = (int)floor(xk);
        k = min(max(k, 0), ntab - 2);
        T s = xk - T(k);
        return (T(1) - s) * dadom[k] + s * dadom[k + 1];
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
template <class T>
void launch_fvjp_paintgrad(Parts<T> p, SortBufs s, Geo g, const T* rhobar, T mass, const T* xbc,
                           T H, int mode, T dr, T k2, T d0, T gp0, T* xbar_out, const T* pbar_in,
                           T* pbar_out, T* sb0, T* sb1, T* sb2, double* dots, hipStream_t st);
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

}  // namespace ml
