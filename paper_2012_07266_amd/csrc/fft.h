// Host entry points of the LDS-staged FFT passes (see fft.hip).
#pragma once
#include "common.h"
#include "paint_halo.h"

namespace ml {

struct PtrTriple {
    void* p[3];
};

// Pencils of length N of a strided pass: element n of pencil w of workgroup
// g sits at base(g) + n*C + w (base = (g / (C/W)) * N*C + (g % (C/W)) * W),
// or at g*W*N + w*N + n when contig; n_wg workgroups.
struct ViewDesc {
    void* ptr;
    long C;
    int contig;
    int n_wg;
};

// true when an n^3 mesh can be transformed in precision T
template <class T> bool fft_supported(int n);

// r2c along axis 2 of an n^3 real mesh, in place: io holds n*n rows of n reals
// on input and n*n rows of n/2 complex (k2 < n/2) on output; nyq gets the
// k2 = n/2 plane [n][n].  tw_h: exp(-2 pi i t/(n/2)), t < n/2;
// tw_post: exp(-2 pi i k/n), k <= n/2.
// `hm`: paint-box shells to merge into the rows while loading (none by
// default).
template <class T>
void fft_r2c_rows(int n, T* io, cx<T>* nyq, const cx<T>* tw_h, const cx<T>* tw_post,
                  hipStream_t st, HaloMerge<T> hm = HaloMerge<T>());
// Unnormalised c2r along axis 2, in place (inverse of fft_r2c_rows times n).
// mul_k2: multiply the spectrum by n2 = k2 first (zero on the nyq plane).
template <class T>
void fft_c2r_rows(int n, T* io, const cx<T>* nyq, const cx<T>* tw_h, const cx<T>* tw_post,
                  hipStream_t st, bool mul_k2 = false);
// c2c along axis 1 (sign +1 forward, -1 unnormalised inverse) on main and nyq.
template <class T>
void fft_c2c_axis1(int n, int sign, cx<T>* main, cx<T>* nyq, const cx<T>* tw, hipStream_t st);
// Unnormalised inverse c2c along axis 1 with two outputs from H = (main,
// nyq): IFFT1(n1 H) in place (zero where |n1| = n/2) and IFFT1(H) into
// (main2, nyq2).
template <class T>
void fft_c2c_axis1_dual(int n, cx<T>* main, cx<T>* nyq, cx<T>* main2, cx<T>* nyq2, const cx<T>* tw,
                        hipStream_t st);
// c2c along axis 0 on main and nyq.
template <class T>
void fft_c2c_axis0(int n, int sign, cx<T>* main, cx<T>* nyq, const cx<T>* tw, hipStream_t st);
// Fused axis-0 pass: forward, h = i G(|n|^2) X, then inverse of n0 h (zero
// where |n0| = n/2) into out[0] and inverse of h into out[1] (out[2] is not
// used).  G(q) is the table G[q], or gscale / q when G is NULL (q > 0;
// G(0) = 0).  Followed by fft_c2c_axis1 on out[0], fft_c2c_axis1_dual on
// out[1] (-> out[1], out[2]) and fft_c2r_rows on the three, the last with
// mul_k2, this yields the three gradient components i n_j G X.
template <class T>
void fft_grad_axis0(int n, cx<T>* main_in, cx<T>* nyq_in, PtrTriple out_main, PtrTriple out_nyq,
                    const cx<T>* tw, const T* G, T gscale, hipStream_t st);

// Transposed fused pass: forward FFT of three spectra along axis 0,
// Y = -i G(|n|^2) sum_j n_j X_j (component j zero where |n_j| = n/2), inverse,
// one output (may alias input 0).
template <class T>
void fft_div_axis0(int n, PtrTriple in_main, PtrTriple in_nyq, cx<T>* out_main, cx<T>* out_nyq,
                   const cx<T>* tw, const T* G, T gscale, hipStream_t st);

}  // namespace ml
