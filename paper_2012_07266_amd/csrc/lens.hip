// Born lightcone projection on gfx950.
//
// The convergence of a source plane at comoving distance chi_s is the
// integral of (3/2) Om (H0/c)^2 q(chi) delta / a along the line of sight with
// q = chi (chi_s - chi) / chi_s (convergence equation of the paper's notation
// section).  With the particles of one PM step standing in for the density
// of its distance shell, every particle image r = x + n L - O (observer O at
// (L/2, L/2, 0), line of sight along axis 2, chi = r_2, theta = r_perp/chi)
// adds  wbase (chi_s - chi) / (chi_s chi a(chi))  to the map, bilinearly, and
// the shell's mean term is added to every pixel by a second kernel.  The
// replica range of each particle is computed directly from the shell depth
// and the field of view, so the work is proportional to the images that
// land on the map.
#include "particles.h"

namespace ml {

constexpr int LB = 256;

template <class T>
__device__ __forceinline__ T a_of_chi(const LensArgs<T>& la, T chi) {
    // cubic Hermite interpolation of a(chi) with exact slopes da/dchi
    T xk = chi / la.dchi;
    int k = (int)floor(xk);
    k = min(max(k, 0), la.ntab - 2);
    T s = xk - T(k);
    T a0 = la.atab[2 * k], d0 = la.atab[2 * k + 1] * la.dchi;
    T a1 = la.atab[2 * k + 2], d1 = la.atab[2 * k + 3] * la.dchi;
    T s2 = s * s, s3 = s2 * s;
    return (T(2) * s3 - T(3) * s2 + T(1)) * a0 + (s3 - T(2) * s2 + s) * d0 +
           (T(3) * s2 - T(2) * s3) * a1 + (s3 - s2) * d1;
}

template <class T>
__device__ __forceinline__ void splat(T* map, int npix, T t0, T t1, T w) {
    T fl0 = floor(t0), fl1 = floor(t1);
    int j0 = (int)fl0, j1 = (int)fl1;
    T f0 = t0 - fl0, f1 = t1 - fl1;
    T wa[2] = {T(1) - f0, f0}, wb[2] = {T(1) - f1, f1};
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        int r = j0 + a;
        if (r < 0 || r >= npix) continue;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            int c = j1 + b;
            if (c < 0 || c >= npix) continue;
            unsafeAtomicAdd(&map[(long)r * npix + c], w * wa[a] * wb[b]);
        }
    }
}

template <class T>
__global__ __launch_bounds__(LB) void k_lens(Parts<T> p, Geo g, LensArgs<T> la, T* kappa) {
    const long n = g.npart;
    const T nmf = T(g.nm);
    const T half = T(0.5) * nmf;
    const T cnear = la.chi_near / la.cell, cfar = la.chi_far / la.cell;  // cells
    const T tmax = T(0.5) * T(la.npix) + T(0.5);   // |theta|/dtheta bound incl. one pixel
    const T hp = T(0.5) * T(la.npix) - T(0.5);
    const long npix2 = (long)la.npix * la.npix;
    T chi_max_src = la.chi_src[0];
    for (int s = 1; s < la.nsrc; ++s) chi_max_src = max(chi_max_src, la.chi_src[s]);
    for (long k = blockIdx.x * (long)LB + threadIdx.x; k < n; k += (long)gridDim.x * LB) {
        int i[3];
        lattice_of_l(p.id[k], g.np, i);
        T u[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            int c;
            T f;
            T v = T(0.5) + p.disp[a * n + k];
            T fl = floor(v);
            f = v - fl;
            c = pmod(g.B * i[a] + (int)fl, g.nm);
            u[a] = T(c) + f;
        }
        if (!(isfinite(u[0]) && isfinite(u[1]) && isfinite(u[2]))) continue;
        int nz0 = (int)floor((cnear - u[2]) / nmf);
        int nz1 = (int)floor((cfar - u[2]) / nmf) + 1;
        for (int nz = nz0; nz <= nz1; ++nz) {
            T rz = u[2] + T(nz) * nmf;
            if (!(rz > cnear && rz <= cfar && rz > T(0))) continue;
            T chi = rz * la.cell;
            if (chi >= chi_max_src) continue;
            T inv = la.inv_dtheta / rz;  // pixels per cell at this distance
            T rmax = tmax / inv;          // |r_perp| bound in cells
            int nx0 = (int)floor((-rmax - u[0] + half) / nmf);
            int nx1 = (int)floor((rmax - u[0] + half) / nmf) + 1;
            int ny0 = (int)floor((-rmax - u[1] + half) / nmf);
            int ny1 = (int)floor((rmax - u[1] + half) / nmf) + 1;
            T ach = a_of_chi(la, chi);
            T base = la.wbase / (chi * ach);
            for (int nx = nx0; nx <= nx1; ++nx) {
                T t0 = (u[0] + T(nx) * nmf - half) * inv + hp;
                if (!(t0 > T(-1) && t0 < T(la.npix))) continue;
                for (int ny = ny0; ny <= ny1; ++ny) {
                    T t1 = (u[1] + T(ny) * nmf - half) * inv + hp;
                    if (!(t1 > T(-1) && t1 < T(la.npix))) continue;
                    for (int s = 0; s < la.nsrc; ++s) {
                        T cs = la.chi_src[s];
                        if (chi < cs) splat(kappa + s * npix2, la.npix, t0, t1, base * (cs - chi) / cs);
                    }
                }
            }
        }
    }
}

template <class T>
void launch_lens(Parts<T> p, Geo g, const LensArgs<T>& la, T* kappa, hipStream_t st) {
    long blocks = (g.npart + LB - 1) / LB;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_lens<T>, dim3(blocks), dim3(LB), 0, st, p, g, la, kappa);
}

template <class T> struct MapVals { T v[MAX_SRC]; };

template <class T>
__global__ void k_add_maps(T* kappa, long npix2, int nsrc, MapVals<T> mv) {
    long total = npix2 * nsrc;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x)
        kappa[i] += mv.v[i / npix2];
}

template <class T>
void launch_add_maps(T* kappa, int npix, int nsrc, const T* vals, hipStream_t st) {
    MapVals<T> mv;
    for (int s = 0; s < MAX_SRC; ++s) mv.v[s] = s < nsrc ? vals[s] : T(0);
    long npix2 = (long)npix * npix;
    long blocks = (npix2 * nsrc + LB - 1) / LB;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_add_maps<T>, dim3(blocks), dim3(LB), 0, st, kappa, npix2, nsrc, mv);
}

template void launch_lens<float>(Parts<float>, Geo, const LensArgs<float>&, float*, hipStream_t);
template void launch_lens<double>(Parts<double>, Geo, const LensArgs<double>&, double*, hipStream_t);
template void launch_add_maps<float>(float*, int, int, const float*, hipStream_t);
template void launch_add_maps<double>(double*, int, int, const double*, hipStream_t);

}  // namespace ml
