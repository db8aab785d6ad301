// Derivative kernels of the PM step, the initial conditions and the lens
// projection on gfx950: reverse mode (vector-Jacobian products) and, in
// part 4, forward mode (Jacobian-vector products, tangents).
//
// Force node f = R(x, M(P(x))): P = CIC paint, M = Fourier force operator,
// R = CIC readout.  For a cotangent fbar:
//   xbar += (dR/dx)^T fbar   gather with the CIC derivative on the force meshes
//   Mbar  = paint(fbar)      three value paints (launch_paint_values)
//   rhobar = M^T Mbar         transposed FFT chain (fft_div_axis0)
//   xbar += mass (dP/dx)^T rhobar
// The CIC derivative is -1 to node floor(u) and +1 to node floor(u)+1 per axis.
// Internally cotangents are in mesh-cell units (H times the Mpc/h ones); the
// caller's arrays are in Mpc/h and lattice order.
#include "adjoint.h"

namespace ml {

constexpr int AB = 512;  // threads per workgroup of the per-tile adjoint kernels

__device__ __forceinline__ int xcd_remap(int b, int nb) {
    if (nb % 8) return b;
    return (b % 8) * (nb / 8) + b / 8;
}

template <class T>
__device__ __forceinline__ void cic_setup(const Geo& g, uint32_t id, const T* d, int ox, int oy,
                                          int oz, int& base, T w[3][2]) {
    int li[3];
    lattice_of_l(id, g.np, li);
    int l[3];
    const int o[3] = {ox, oy, oz};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        T v = T(0.5) + d[a];
        T fl = floor(v);
        T t = v - fl;
        int c = g.B * li[a] + (int)fl;
        if ((unsigned)c >= (unsigned)g.nm) c = pmod(c, g.nm);
        l[a] = min(max(c - o[a], 0), TILE - 1);
        w[a][0] = T(1) - t;
        w[a][1] = t;
    }
    base = (l[0] * TE + l[1]) * TE + l[2];
}

// value and gradient (d/du) of the CIC interpolation of an LDS tile
template <class T>
__device__ __forceinline__ void cic_grad(const T* ft, int base, const T w[3][2], T& val, T gr[3]) {
    val = T(0);
    gr[0] = gr[1] = gr[2] = T(0);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                T m = ft[base + (a * TE + b) * TE + c];
                T d0 = a ? T(1) : T(-1), d1 = b ? T(1) : T(-1), d2 = c ? T(1) : T(-1);
                val += w[0][a] * w[1][b] * w[2][c] * m;
                gr[0] += d0 * w[1][b] * w[2][c] * m;
                gr[1] += w[0][a] * d1 * w[2][c] * m;
                gr[2] += w[0][a] * w[1][b] * d2 * m;
            }
}

// Workgroup reductions with one atomic per workgroup (same-address atomics
// from every wave serialise).  Every thread of the workgroup must call them;
// red is LDS scratch of NT / 64 entries, reusable across calls.
template <int NT>
__device__ __forceinline__ void block_add(double* dst, double v, double* red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    __syncthreads();  // a previous call may still be reading red
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < NT / 64; ++i) t += red[i];
        if (t != 0.0) unsafeAtomicAdd(dst, t);
    }
}
template <int NT>
__device__ __forceinline__ void block_max(uint32_t* dst, float v, float* red) {
    for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < NT / 64; ++i) v = fmaxf(v, red[i]);
        if (v > 0.f) atomicMax(dst, __float_as_uint(v));
    }
}

// Global offset of entry i of a tile's 17^3 box at origin (ox, oy, oz),
// periodic.
__device__ __forceinline__ long tile_offset(int i, int nm, int ox, int oy, int oz) {
    const int x = i / (TE * TE), y = (i / TE) % TE, z = i % TE;
    int gx = ox + x, gy = oy + y, gz = oz + z;
    if (gx >= nm) gx -= nm;
    if (gy >= nm) gy -= nm;
    if (gz >= nm) gz -= nm;
    return ((long)gx * nm + gy) * nm + gz;
}

// Stage the 17^3 boxes of NM meshes into LDS.  Every load of the batch is
// issued before the first LDS store (slots past the box repeat its last
// entry and are not stored): a loop that stores each value as it arrives
// waits for every load in turn.
template <class T, int NM>
__device__ __forceinline__ void stage_tiles(T (*ft)[TE * TE * TE], const T* const (&mesh)[NM],
                                            int nm, int ox, int oy, int oz, int tid) {
    constexpr int TC = TE * TE * TE;
    constexpr int IT = (TC + AB - 1) / AB;
    T v[NM][IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        int i = tid + it * AB;
        i = i < TC ? i : TC - 1;
        const long c = tile_offset(i, nm, ox, oy, oz);
#pragma unroll
        for (int m = 0; m < NM; ++m) v[m][it] = mesh[m][c];
    }
    issue_fence();
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int i = tid + it * AB;
        if (i < TC) {
#pragma unroll
            for (int m = 0; m < NM; ++m) ft[m][i] = v[m][it];
        }
    }
}

// ---------------------------------------------------------------------------
// 1. readout part of the force-node VJP
// ---------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(AB) void k_fvjp_readout(Parts<T> p, SortBufs s, Geo g, const T* f0,
                                                     const T* f1, const T* f2, const T* xbar_in,
                                                     const T* pbar_in, T H, T ckick, T* xbc,
                                                     T* fbc, double* dots, uint32_t* fmax_bits) {
    constexpr int TC = TE * TE * TE;
    __shared__ T ft[3][TC];
    __shared__ double red[AB / 64];
    __shared__ float redf[AB / 64];
    const int tid = threadIdx.x;
    const int t = xcd_remap(blockIdx.x, gridDim.x);
    const int tx = t / (g.nt * g.nt), ty = (t / g.nt) % g.nt, tz = t % g.nt;
    const int ox = tx * TILE, oy = ty * TILE, oz = tz * TILE;
    const int b0 = tile_block(g, tx, ty, tz);
    const uint32_t lo = s.start[b0], hi = s.start[b0 + BPT];
    if (lo == hi) return;
    {
        const T* const fm[3] = {f0, f1, f2};
        stage_tiles<T, 3>(ft, fm, g.nm, ox, oy, oz, tid);
    }
    __syncthreads();
    const long n = g.npart;
    double dot = 0.0;
    float fmax = 0.f;
    for (uint32_t k0 = lo; k0 < hi; k0 += AB) {
        uint32_t k = k0 + tid;
        if (k < hi) {
            uint32_t id = p.id[k];
            long L = lattice_index(id, g.np);
            T d[3] = {p.disp[k], p.disp[n + k], p.disp[2 * n + k]};
            int base;
            T w[3][2];
            cic_setup(g, id, d, ox, oy, oz, base, w);
            T xb[3], fb[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                T pb = H * pbar_in[a * n + L];
                xb[a] = H * xbar_in[a * n + L];
                fb[a] = ckick * pb;
                dot += (double)pb * (double)p.acc[a * n + k];
                fmax = fmaxf(fmax, fabsf((float)fb[a]));
            }
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                T val, gr[3];
                cic_grad(ft[j], base, w, val, gr);
#pragma unroll
                for (int a = 0; a < 3; ++a) xb[a] += fb[j] * gr[a];
            }
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                xbc[a * n + k] = xb[a];
                fbc[a * n + k] = fb[a];
            }
        }
    }
    block_add<AB>(&dots[0], dot, red);
    block_max<AB>(fmax_bits, fmax, redf);
}

// ---------------------------------------------------------------------------
// 2. paint part of the force-node VJP, then the drift reverse (mode 0) or the
//    initial-condition cotangent (mode 1)
// ---------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(AB) void k_fvjp_paintgrad(Parts<T> p, SortBufs s, Geo g,
                                                       const T* rhobar, T mass, const T* xbc,
                                                       T H, int mode, T dr, T k2, T d0, T gp0,
                                                       T* xbar_out, const T* pbar_in, T* pbar_out,
                                                       const T* phbar, T* sb0, T* sb1, T* sb2,
                                                       double* dots) {
    constexpr int TC = TE * TE * TE;
    __shared__ T ft[1][TC];
    __shared__ double red[AB / 64];
    const int tid = threadIdx.x;
    const int t = xcd_remap(blockIdx.x, gridDim.x);
    const int tx = t / (g.nt * g.nt), ty = (t / g.nt) % g.nt, tz = t % g.nt;
    const int ox = tx * TILE, oy = ty * TILE, oz = tz * TILE;
    const int b0 = tile_block(g, tx, ty, tz);
    const uint32_t lo = s.start[b0], hi = s.start[b0 + BPT];
    if (lo == hi) return;
    {
        const T* const fm[1] = {rhobar};
        stage_tiles<T, 1>(ft, fm, g.nm, ox, oy, oz, tid);
    }
    __syncthreads();
    const long n = g.npart;
    double a1 = 0.0, a2 = 0.0, a3 = 0.0;
    for (uint32_t k0 = lo; k0 < hi; k0 += AB) {
        uint32_t k = k0 + tid;
        if (k < hi) {
            uint32_t id = p.id[k];
            long L = lattice_index(id, g.np);
            T d[3] = {p.disp[k], p.disp[n + k], p.disp[2 * n + k]};
            int base;
            T w[3][2];
            cic_setup(g, id, d, ox, oy, oz, base, w);
            T val, gr[3];
            cic_grad(ft[0], base, w, val, gr);
            T xb[3], pb[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                xb[a] = xbc[a * n + k] + mass * gr[a];
                pb[a] = H * pbar_in[a * n + L];
            }
            if (mode == 0) {
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    T ph = p.mom[a * n + k] - k2 * p.acc[a * n + k];
                    a1 += (double)xb[a] * (double)ph;
                    xbar_out[a * n + L] = xb[a] / H;
                    pbar_out[a * n + L] = (pb[a] + dr * xb[a]) / H + (phbar ? phbar[a * n + L] : T(0));
                }
            } else {
                T* sbo[3] = {sb0, sb1, sb2};
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    T sv = p.mom[a * n + k] / gp0;
                    T sbar = d0 * xb[a] + gp0 * pb[a];
                    a1 += (double)xb[a] * (double)sv;
                    a2 += (double)pb[a] * (double)sv;
                    a3 += (double)sbar * (double)sv;
                    sbo[a][k] = sbar;  // tile-sorted order
                }
            }
        }
    }
    block_add<AB>(&dots[1], a1, red);
    if (mode == 1) {
        block_add<AB>(&dots[2], a2, red);
        block_add<AB>(&dots[3], a3, red);
    }
}

template <class T>
__global__ __launch_bounds__(256) void k_dot3(const T* a0, const T* a1, const T* a2, const T* b0,
                                              const T* b1, const T* b2, long n, double* dst) {
    __shared__ double red[4];
    double acc = 0.0;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        acc += (double)a0[i] * b0[i] + (double)a1[i] * b1[i] + (double)a2[i] * b2[i];
    block_add<256>(dst, acc, red);
}

// sum_k sum_j sorted[j][k] * lattice_j[L(k)]
template <class T>
__global__ __launch_bounds__(256) void k_dot_sorted_lattice(Parts<T> p, Geo g, const T* sorted,
                                                            const T* l0, const T* l1, const T* l2,
                                                            double* dst) {
    __shared__ double red[4];
    const long n = g.npart;
    double acc = 0.0;
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
        long L = lattice_index(p.id[k], g.np);
        acc += (double)sorted[k] * l0[L] + (double)sorted[n + k] * l1[L] +
               (double)sorted[2 * n + k] * l2[L];
    }
    block_add<256>(dst, acc, red);
}

// lattice_j[L(k)] = sorted[j][k]
template <class T>
__global__ void k_sorted_to_lattice(Parts<T> p, Geo g, const T* sorted, T* l0, T* l1, T* l2) {
    const long n = g.npart;
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
        long L = lattice_index(p.id[k], g.np);
        l0[L] = sorted[k];
        l1[L] = sorted[n + k];
        l2[L] = sorted[2 * n + k];
    }
}

template <class T>
__global__ __launch_bounds__(256) void k_map_sums(const T* kbar, long npix2, int nsrc, double* dst) {
    __shared__ double red[4];
    for (int s = 0; s < nsrc; ++s) {
        double acc = 0.0;
        for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < npix2; i += (long)gridDim.x * blockDim.x)
            acc += (double)kbar[(long)s * npix2 + i];
        block_add<256>(&dst[s], acc, red);
    }
}

// ---------------------------------------------------------------------------
// 3. lens projection VJP: per particle, per image, gather of kbar and its
//    gradient; position cotangent accumulated in registers, one write per
//    particle (no atomics); Omega_m part of the weights reduced.
// ---------------------------------------------------------------------------
// Cubic Hermite interpolant of a (value, d/dchi) table on the chi grid, and
// its derivative: the interpolation the projection uses.
template <class T>
__device__ __forceinline__ void tab_interp(const T* tab, const LensArgs<T>& la, T chi, T& a,
                                           T& dadchi) {
    T xk = chi / la.dchi;
    int k = (int)floor(xk);
    k = min(max(k, 0), la.ntab - 2);
    T s = xk - T(k);
    T a0 = tab[2 * k], m0 = tab[2 * k + 1] * la.dchi;
    T a1 = tab[2 * k + 2], m1 = tab[2 * k + 3] * la.dchi;
    T s2 = s * s, s3 = s2 * s;
    a = (T(2) * s3 - T(3) * s2 + T(1)) * a0 + (s3 - T(2) * s2 + s) * m0 + (T(3) * s2 - T(2) * s3) * a1 +
        (s3 - s2) * m1;
    T da = (T(6) * s2 - T(6) * s) * a0 + (T(3) * s2 - T(4) * s + T(1)) * m0 +
           (T(6) * s - T(6) * s2) * a1 + (T(3) * s2 - T(2) * s) * m1;
    dadchi = da / la.dchi;
}

template <class T>
__device__ __forceinline__ void a_interp(const LensArgs<T>& la, T chi, T& a, T& dadchi) {
    tab_interp(la.atab, la, chi, a, dadchi);
}

template <class T>
__device__ __forceinline__ void bilinear_grad(const T* km, int npix, T t0, T t1, T& v, T& g0, T& g1) {
    T fl0 = floor(t0), fl1 = floor(t1);
    int j0 = (int)fl0, j1 = (int)fl1;
    T f0 = t0 - fl0, f1 = t1 - fl1;
    v = g0 = g1 = T(0);
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        int r = j0 + a;
        if (r < 0 || r >= npix) continue;
        T w0 = a ? f0 : T(1) - f0, d0 = a ? T(1) : T(-1);
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            int c = j1 + b;
            if (c < 0 || c >= npix) continue;
            T w1 = b ? f1 : T(1) - f1, d1 = b ? T(1) : T(-1);
            T m = km[(long)r * npix + c];
            v += w0 * w1 * m;
            g0 += d0 * w1 * m;
            g1 += w0 * d1 * m;
        }
    }
}

// Position cotangent (in the image frame) and Omega_m term of one image at
// (rx, ry, rz) cells from the observer, rz in the shell and chi = rz cell.
template <class T>
__device__ __forceinline__ void lens_vjp_image(const LensArgs<T>& la, const LensVjpArgs<T>& lv,
                                               const T* kbar, long npix2, T rx, T ry, T rz, T chi,
                                               T a, T dadchi, T dadom, T hp, T dth, T& gx,
                                               T& gy, T& gz, double& om_acc) {
    const T inv = la.inv_dtheta / rz;
    const T t0 = rx * inv + hp, t1 = ry * inv + hp;
    if (!(t0 > T(-1) && t0 < T(la.npix) && t1 > T(-1) && t1 < T(la.npix))) return;
    const T rxp = rx * la.cell, ryp = ry * la.cell;  // Mpc/h
    const T invp = T(1) / (chi * dth);
    for (int s = 0; s < la.nsrc; ++s) {
        T cs = la.chi_src[s];
        if (!(chi < cs)) continue;
        T v, g0, g1;
        bilinear_grad(kbar + s * npix2, la.npix, t0, t1, v, g0, g1);
        T gs = (cs - chi) / (cs * chi * a);
        T w = la.wbase * gs;
        T dg = -T(1) / (cs * chi * a) - gs / chi - gs * dadchi / a;
        T dw = la.wbase * dg;
        gx += w * g0 * invp;
        gy += w * g1 * invp;
        gz += dw * v - w * (g0 * rxp + g1 * ryp) * invp / chi;
        T dwdom = w / lv.omega_m + la.wbase * (lv.dchis_dom[s] / (cs * cs * a) - gs * dadom / a);
        om_acc += (double)dwdom * (double)v;
    }
}

// Cube symmetries of the replicas (the hash and tables of the projection).
__device__ __forceinline__ unsigned long long vjp_mix64(unsigned long long z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__device__ __forceinline__ int vjp_replica_symmetry(int nx, int ny, int nz, unsigned long long seed) {
    const unsigned long long u = ((unsigned long long)(nx + (1 << 20)) << 42) |
                                 ((unsigned long long)(ny + (1 << 20)) << 21) |
                                 (unsigned long long)(nz + (1 << 20));
    return (int)(vjp_mix64(seed ^ vjp_mix64(u)) % 48ull);
}
__device__ __forceinline__ int vjp_sym_axis(int s, int j) {
    const int p = s >> 3, f = p >> 1;
    const int r0 = f == 0 ? 1 : 0, r1 = f == 2 ? 1 : 2;
    return j == 0 ? f : (j == 1 ? ((p & 1) ? r1 : r0) : ((p & 1) ? r0 : r1));
}

template <class T>
__global__ __launch_bounds__(256) void k_lens_vjp(Parts<T> p, Geo g, LensArgs<T> la, LensVjpArgs<T> lv,
                                                  const T* kbar, T* xbar, double* dots) {
    __shared__ double red[4];
    const long n = g.npart;
    const T nmf = T(g.nm), half = T(0.5) * nmf;
    const T cnear = la.chi_near / la.cell, cfar = la.chi_far / la.cell;
    const T tmax = T(0.5) * T(la.npix) + T(0.5);
    const T hp = T(0.5) * T(la.npix) - T(0.5);
    const T dth = T(1) / la.inv_dtheta;
    const long npix2 = (long)la.npix * la.npix;
    T chi_max_src = la.chi_src[0];
    for (int s = 1; s < la.nsrc; ++s) chi_max_src = max(chi_max_src, la.chi_src[s]);
    double om_acc = 0.0;
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
        uint32_t id = p.id[k];
        int li[3];
        lattice_of_l(id, g.np, li);
        T u[3];
        int cz = 0;   // axis 2 as an integer cell and a fraction (membership)
        T fz = T(0);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            T v = T(0.5) + p.disp[a * n + k];
            T fl = floor(v);
            int c = g.B * li[a] + (int)fl;
            if ((unsigned)c >= (unsigned)g.nm) c = pmod(c, g.nm);
            u[a] = T(c) + (v - fl);
            if (a == 2) {
                cz = c;
                fz = v - fl;
            }
        }
        if (!(isfinite(u[0]) && isfinite(u[1]) && isfinite(u[2]))) continue;
        T gx = 0, gy = 0, gz = 0;
        T qx = 0, qy = 0, qz = 0;  // drift-momentum cotangent (sub-evolution)
        if (la.rot || la.sub) {
            // the step's drift momentum (cells) and the largest move it
            // makes within the shell: |dr| <= the step's drift factor
            T ph[3] = {T(0), T(0), T(0)};
            T margin = T(0);
            if (la.sub) {
#pragma unroll
                for (int a = 0; a < 3; ++a) ph[a] = p.mom[a * n + k] - la.sub_k2 * p.acc[a * n + k];
                margin = min(la.sub_dr * max(max(fabs(ph[0]), fabs(ph[1])), fabs(ph[2])), nmf);
            }
            // every replica whose box can reach the shell and the map: an
            // image's end-of-step depth in replica nz lies in [nz Nm, (nz + 1) Nm]
            const int mz0 = max((int)floor(cnear / nmf), 0), mz1 = (int)floor(cfar / nmf);
            for (int nz = mz0; nz <= mz1; ++nz) {
                const T rz_hi = min(T(nz + 1) * nmf, cfar) + margin;
                const T rmax = tmax * rz_hi / la.inv_dtheta + margin;
                const int mx0 = (int)floor((-rmax + half) / nmf) - 1;
                const int mx1 = (int)floor((rmax + half) / nmf);
                for (int nx = mx0; nx <= mx1; ++nx)
                    for (int ny = mx0; ny <= mx1; ++ny) {
                        const int sym = la.rot ? vjp_replica_symmetry(nx, ny, nz, la.rot_seed) : 0;
                        T ui[3], pi[3];
#pragma unroll
                        for (int j = 0; j < 3; ++j) {
                            const int ax = vjp_sym_axis(sym, j);
                            const T c = ax == 0 ? u[0] : (ax == 1 ? u[1] : u[2]);
                            const T q = ax == 0 ? ph[0] : (ax == 1 ? ph[1] : ph[2]);
                            const bool fl = (sym >> j) & 1;
                            ui[j] = fl ? nmf - c : c;
                            pi[j] = fl ? -q : q;
                        }
                        T rx = ui[0] + T(nx) * nmf - half, ry = ui[1] + T(ny) * nmf - half;
                        T rz = ui[2] + T(nz) * nmf;
                        int cr = cz;
                        T fr = fz;
                        if (sym) split_cell(ui[2], cr, fr);
                        if (!depth_in_shell(cr, fr, zbound<T>(la.cnear_d, nz, g.nm),
                                            zbound<T>(la.cfar_d, nz, g.nm)) ||
                            !(rz > T(0)))
                            continue;
                        T dr = T(0), ddr = T(0), de = T(0);
                        T chi_e = rz * la.cell;
                        if (la.sub) {
                            // along the step's drift to a(chi) of the
                            // end-of-step depth
                            T dd;
                            tab_interp(la.dtab, la, chi_e, de, dd);
                            dr = (de - la.d_end) * la.sub_scale;
                            ddr = dd * la.sub_scale;  // d dr / d chi_e, per Mpc/h
                            rx += dr * pi[0];
                            ry += dr * pi[1];
                            rz += dr * pi[2];
                            if (!(rz > T(0))) continue;
                        }
                        const T chi = rz * la.cell;
                        if (chi >= chi_max_src) continue;
                        T a, dadchi;
                        a_interp(la, chi, a, dadchi);
                        T hx = 0, hy = 0, hz = 0;
                        double om_img = 0.0;
                        lens_vjp_image(la, lv, kbar, npix2, rx, ry, rz, chi, a, dadchi,
                                       lv.dadom_at(chi), hp, dth, hx, hy, hz, om_img);
                        om_acc += om_img;
                        T ix = hx, iy = hy, iz = hz;
                        if (la.sub) {
                            // r' = r + dr(chi_e) p_h: the depth also moves dr
                            const T gp = (hx * pi[0] + hy * pi[1] + hz * pi[2]) * la.cell;
                            iz += ddr * gp;
                            const T ddr_dom = (lv.ddom_at(chi_e) - lv.dd_end_dom) * la.sub_scale +
                                              (de - la.d_end) * lv.dscale_dom;
                            om_acc += (double)gp * (double)ddr_dom;
                        }
                        // back to the box frame: image axis j is box axis
                        // vjp_sym_axis(sym, j), reflected when flip j is set
#pragma unroll
                        for (int j = 0; j < 3; ++j) {
                            T v = j == 0 ? ix : (j == 1 ? iy : iz);
                            T w = j == 0 ? hx : (j == 1 ? hy : hz);
                            if ((sym >> j) & 1) {
                                v = -v;
                                w = -w;
                            }
                            w *= dr;
                            const int ax = vjp_sym_axis(sym, j);
                            gx += ax == 0 ? v : T(0);
                            gy += ax == 1 ? v : T(0);
                            gz += ax == 2 ? v : T(0);
                            qx += ax == 0 ? w : T(0);
                            qy += ax == 1 ? w : T(0);
                            qz += ax == 2 ? w : T(0);
                        }
                    }
            }
        } else {
        int nz0 = (int)floor((cnear - u[2]) / nmf);
        int nz1 = (int)floor((cfar - u[2]) / nmf) + 1;
        for (int nz = nz0; nz <= nz1; ++nz) {
            T rz = u[2] + T(nz) * nmf;
            if (!depth_in_shell(cz, fz, zbound<T>(la.cnear_d, nz, g.nm),
                                zbound<T>(la.cfar_d, nz, g.nm)) ||
                !(rz > T(0)))
                continue;
            T chi = rz * la.cell;
            if (chi >= chi_max_src) continue;
            T inv = la.inv_dtheta / rz;
            T rmax = tmax / inv;
            int nx0 = (int)floor((-rmax - u[0] + half) / nmf), nx1 = (int)floor((rmax - u[0] + half) / nmf) + 1;
            int ny0 = (int)floor((-rmax - u[1] + half) / nmf), ny1 = (int)floor((rmax - u[1] + half) / nmf) + 1;
            T a, dadchi;
            a_interp(la, chi, a, dadchi);
            T dadom = lv.dadom_at(chi);
            for (int nx = nx0; nx <= nx1; ++nx) {
                T rx = (u[0] + T(nx) * nmf - half);  // cells
                T t0 = rx * inv + hp;
                if (!(t0 > T(-1) && t0 < T(la.npix))) continue;
                for (int ny = ny0; ny <= ny1; ++ny) {
                    T ry = (u[1] + T(ny) * nmf - half);
                    T t1 = ry * inv + hp;
                    if (!(t1 > T(-1) && t1 < T(la.npix))) continue;
                    T rxp = rx * la.cell, ryp = ry * la.cell;  // Mpc/h
                    T invp = T(1) / (chi * dth);
                    for (int s = 0; s < la.nsrc; ++s) {
                        T cs = la.chi_src[s];
                        if (!(chi < cs)) continue;
                        T v, g0, g1;
                        bilinear_grad(kbar + s * npix2, la.npix, t0, t1, v, g0, g1);
                        T gs = (cs - chi) / (cs * chi * a);
                        T w = la.wbase * gs;
                        T dg = -T(1) / (cs * chi * a) - gs / chi - gs * dadchi / a;
                        T dw = la.wbase * dg;
                        gx += w * g0 * invp;
                        gy += w * g1 * invp;
                        gz += dw * v - w * (g0 * rxp + g1 * ryp) * invp / chi;
                        T dwdom = w / lv.omega_m +
                                  la.wbase * (lv.dchis_dom[s] / (cs * cs * a) - gs * dadom / a);
                        om_acc += (double)dwdom * (double)v;
                    }
                }
            }
        }
        }
        if (gx != T(0) || gy != T(0) || gz != T(0)) {
            long L = lattice_index(id, g.np);
            xbar[L] += gx;
            xbar[n + L] += gy;
            xbar[2 * n + L] += gz;
        }
        if (la.sub && (qx != T(0) || qy != T(0) || qz != T(0))) {
            long L = lattice_index(id, g.np);
            lv.phbar[L] += qx;
            lv.phbar[n + L] += qy;
            lv.phbar[2 * n + L] += qz;
        }
    }
    block_add<256>(&dots[4], om_acc, red);
}

// ---------------------------------------------------------------------------
// 4. forward-mode tangents (Jacobian-vector products).  The tangent state
//    (x_dot, p_dot, f_dot) is kept in tile order, in Mpc/h, and travels with
//    the particles through the sort, so every access here is coalesced.
// ---------------------------------------------------------------------------
// y = a y + b x (y is not read when a == 0)
template <class T>
__global__ void k_lin(T* y, const T* x, T a, T b, long n) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        y[i] = (a == T(0) ? T(0) : a * y[i]) + b * x[i];
}

// Initial-condition tangent from the displacement tangent t and the
// displacement s (lattice order, cells): x_dot = H (D t + cD s),
// p_dot = H (gp t + cgp s).  t may alias x_dot.
template <class T>
__global__ void k_ic_tangent(const T* t0, const T* t1, const T* t2, const T* s0, const T* s1,
                             const T* s2, T* xd, T* pd, T D, T gp, T cD, T cgp, T H, long n) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const T t[3] = {t0[i], t1[i], t2[i]};
        const T sv[3] = {s0[i], s1[i], s2[i]};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            xd[a * n + i] = H * (D * t[a] + cD * sv[a]);
            pd[a * n + i] = H * (gp * t[a] + cgp * sv[a]);
        }
    }
}

// sorted[a][k] = lattice[a][L(k)]
template <class T>
__global__ void k_lattice_to_sorted(Parts<T> p, Geo g, const T* lat, T* sorted) {
    const long n = g.npart;
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
        const long L = lattice_index(p.id[k], g.np);
#pragma unroll
        for (int a = 0; a < 3; ++a) sorted[a * n + k] = lat[a * n + L];
    }
}

// Tangent of the first half-kick and the drift of a step, at the state
// before it (force f = acc at x):
//   ph_dot = p_dot + K1 f_dot + cK1 f,   x_dot += Dr ph_dot + cDr (p + K1 f)
// with cK1, cDr the Omega_m tangent times dK1/dOm, dDr/dOm.  In place.
template <class T>
__global__ void k_jvp_pre(Parts<T> p, Geo g, T* xdot, T* pdot, const T* fdot, T H, T k1, T dr,
                          T ck1, T cdr) {
    const long n = g.npart;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < 3 * n; i += (long)gridDim.x * blockDim.x) {
        const T f = H * p.acc[i];
        const T ph = H * p.mom[i] + k1 * f;
        const T phd = pdot[i] + k1 * fdot[i] + ck1 * f;
        xdot[i] += dr * phd + cdr * ph;
        pdot[i] = phd;
    }
}

// Readout part of the force tangent: f_dot_j = u_dot . grad R(x, M_j) on the
// force meshes M_j of the current state, into fbc (cells), u_dot = x_dot / H;
// and a bound of mass sum_a |u_dot_a| (the tangent paint's scale) into
// vmax_bits, one atomic per workgroup.
template <class T>
__global__ __launch_bounds__(AB) void k_fjvp_gather(Parts<T> p, SortBufs s, Geo g, const T* f0,
                                                    const T* f1, const T* f2, const T* xdot,
                                                    T invH, T mass, T* fbc,
                                                    uint32_t* vmax_bits) {
    constexpr int TC = TE * TE * TE;
    __shared__ T ft[3][TC];
    __shared__ float redf[AB / 64];
    const int tid = threadIdx.x;
    const int t = xcd_remap(blockIdx.x, gridDim.x);
    const int tx = t / (g.nt * g.nt), ty = (t / g.nt) % g.nt, tz = t % g.nt;
    const int ox = tx * TILE, oy = ty * TILE, oz = tz * TILE;
    const int b0 = tile_block(g, tx, ty, tz);
    const uint32_t lo = s.start[b0], hi = s.start[b0 + BPT];
    if (lo == hi) return;
    {
        const T* const fm[3] = {f0, f1, f2};
        stage_tiles<T, 3>(ft, fm, g.nm, ox, oy, oz, tid);
    }
    __syncthreads();
    const long n = g.npart;
    float vmax = 0.f;
    for (uint32_t k0 = lo; k0 < hi; k0 += AB) {
        uint32_t k = k0 + tid;
        if (k < hi) {
            uint32_t id = p.id[k];
            T d[3] = {p.disp[k], p.disp[n + k], p.disp[2 * n + k]};
            int base;
            T w[3][2];
            cic_setup(g, id, d, ox, oy, oz, base, w);
            T ud[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) ud[a] = invH * xdot[a * n + k];
            vmax = fmaxf(vmax, (float)(mass * (fabs(ud[0]) + fabs(ud[1]) + fabs(ud[2]))));
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                T val, gr[3];
                cic_grad(ft[j], base, w, val, gr);
                fbc[j * n + k] = ud[0] * gr[0] + ud[1] * gr[1] + ud[2] * gr[2];
            }
        }
    }
    // a bound slightly above the maximum keeps float rounding of the bound
    // from under-sizing the fixed-point scale
    block_max<AB>(vmax_bits, vmax * 1.0001f, redf);
}

// Paint part of the force tangent and the second half-kick: with M_dot_j the
// force meshes of the tangent density, f_dot_j = fbc_j + R(x, M_dot_j);
// f_dot (Mpc/h) = H f_dot_j and, if pdot is set, p_dot += H (K2 f_dot_j + cK2 f_j).
template <class T>
__global__ __launch_bounds__(AB) void k_fjvp_readout_kick(Parts<T> p, SortBufs s, Geo g, const T* m0,
                                                          const T* m1, const T* m2, const T* fbc,
                                                          T H, T k2, T ck2, T* pdot, T* fdot) {
    constexpr int TC = TE * TE * TE;
    __shared__ T ft[3][TC];
    const int tid = threadIdx.x;
    const int t = xcd_remap(blockIdx.x, gridDim.x);
    const int tx = t / (g.nt * g.nt), ty = (t / g.nt) % g.nt, tz = t % g.nt;
    const int ox = tx * TILE, oy = ty * TILE, oz = tz * TILE;
    const int b0 = tile_block(g, tx, ty, tz);
    const uint32_t lo = s.start[b0], hi = s.start[b0 + BPT];
    if (lo == hi) return;
    {
        const T* const fm[3] = {m0, m1, m2};
        stage_tiles<T, 3>(ft, fm, g.nm, ox, oy, oz, tid);
    }
    __syncthreads();
    const long n = g.npart;
    for (uint32_t k0 = lo; k0 < hi; k0 += AB) {
        uint32_t k = k0 + tid;
        if (k < hi) {
            uint32_t id = p.id[k];
            T d[3] = {p.disp[k], p.disp[n + k], p.disp[2 * n + k]};
            int base;
            T w[3][2];
            cic_setup(g, id, d, ox, oy, oz, base, w);
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                T val = T(0);
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b)
#pragma unroll
                        for (int c = 0; c < 2; ++c)
                            val += w[0][a] * w[1][b] * w[2][c] * ft[j][base + (a * TE + b) * TE + c];
                const T fd = fbc[j * n + k] + val;
                fdot[j * n + k] = H * fd;
                if (pdot) pdot[j * n + k] += H * (k2 * fd + ck2 * p.acc[j * n + k]);
            }
        }
    }
}

// Tangent of one image's splat: kappa_dot_s += (dw/dchi z_dot + Om_dot
// dw/dOm) B + w (dB/dt0 t0_dot + dB/dt1 t1_dot), t_dot = (r_perp_dot -
// r_perp z_dot / chi) / (chi dtheta), (x_dot, y_dot, z_dot) the position
// tangent in the image frame (Mpc/h).
template <class T>
__device__ __forceinline__ void lens_jvp_image(const LensArgs<T>& la, const LensVjpArgs<T>& lv,
                                               T* kdot, long npix2, T rx, T ry, T rz, T chi, T a,
                                               T dadchi, T dadom, T hp, T dth, T xd, T yd, T zd,
                                               T om_dot) {
    const T inv = la.inv_dtheta / rz;
    const T t0 = rx * inv + hp, t1 = ry * inv + hp;
    if (!(t0 > T(-1) && t0 < T(la.npix) && t1 > T(-1) && t1 < T(la.npix))) return;
    const T rxp = rx * la.cell, ryp = ry * la.cell;  // Mpc/h
    const T invp = T(1) / (chi * dth);
    const T td0 = (xd - rxp * zd / chi) * invp, td1 = (yd - ryp * zd / chi) * invp;
    const T fl0 = floor(t0), fl1 = floor(t1);
    const int j0 = (int)fl0, j1 = (int)fl1;
    const T f0 = t0 - fl0, f1 = t1 - fl1;
    for (int s = 0; s < la.nsrc; ++s) {
        const T cs = la.chi_src[s];
        if (!(chi < cs)) continue;
        const T gs = (cs - chi) / (cs * chi * a);
        const T w = la.wbase * gs;
        const T dg = -T(1) / (cs * chi * a) - gs / chi - gs * dadchi / a;
        const T dwdom = w / lv.omega_m + la.wbase * (lv.dchis_dom[s] / (cs * cs * a) - gs * dadom / a);
        const T c = la.wbase * dg * zd + om_dot * dwdom;
        T* km = kdot + s * npix2;
#pragma unroll
        for (int ia = 0; ia < 2; ++ia) {
            const int r = j0 + ia;
            if (r < 0 || r >= la.npix) continue;
            const T w0 = ia ? f0 : T(1) - f0, d0 = ia ? T(1) : T(-1);
#pragma unroll
            for (int ib = 0; ib < 2; ++ib) {
                const int col = j1 + ib;
                if (col < 0 || col >= la.npix) continue;
                const T w1 = ib ? f1 : T(1) - f1, d1 = ib ? T(1) : T(-1);
                unsafeAtomicAdd(&km[(long)r * la.npix + col],
                                c * w0 * w1 + w * (d0 * w1 * td0 + w0 * d1 * td1));
            }
        }
    }
}

// Lens projection tangent: every image of every particle splats its tangent
// (same image set as the projection and its VJP).  With sub-evolution the
// image moves to r' = r + dr(chi_e) p_h and its tangent to
// r'_dot = r_dot + (d dr / d chi_e) r_dot_z p_h + dr p_h_dot + Om_dot (d dr / dOm) p_h,
// p_h = p - K2 f and p_h_dot = p_dot - K2 f_dot - ck2 f (ck2 = Om_dot dK2/dOm).
template <class T>
__global__ __launch_bounds__(256) void k_lens_jvp(Parts<T> p, Geo g, LensArgs<T> la, LensVjpArgs<T> lv,
                                                  const T* xdot, const T* pdot, const T* fdot,
                                                  T ck2, T om_dot, T* kdot) {
    const long n = g.npart;
    const T nmf = T(g.nm), half = T(0.5) * nmf;
    const T cnear = la.chi_near / la.cell, cfar = la.chi_far / la.cell;
    const T tmax = T(0.5) * T(la.npix) + T(0.5);
    const T hp = T(0.5) * T(la.npix) - T(0.5);
    const T dth = T(1) / la.inv_dtheta;
    const long npix2 = (long)la.npix * la.npix;
    T chi_max_src = la.chi_src[0];
    for (int s = 1; s < la.nsrc; ++s) chi_max_src = max(chi_max_src, la.chi_src[s]);
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
        uint32_t id = p.id[k];
        int li[3];
        lattice_of_l(id, g.np, li);
        T u[3];
        int cz = 0;   // axis 2 as an integer cell and a fraction (membership)
        T fz = T(0);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            T v = T(0.5) + p.disp[a * n + k];
            T fl = floor(v);
            int c = g.B * li[a] + (int)fl;
            if ((unsigned)c >= (unsigned)g.nm) c = pmod(c, g.nm);
            u[a] = T(c) + (v - fl);
            if (a == 2) {
                cz = c;
                fz = v - fl;
            }
        }
        if (!(isfinite(u[0]) && isfinite(u[1]) && isfinite(u[2]))) continue;
        const T xb[3] = {xdot[k], xdot[n + k], xdot[2 * n + k]};
        if (la.rot || la.sub) {
            // drift momentum (cells) and its tangent (Mpc/h), and the largest
            // move within the shell: |dr| <= the step's drift factor
            T ph[3] = {T(0), T(0), T(0)}, phd[3] = {T(0), T(0), T(0)};
            T margin = T(0);
            if (la.sub) {
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const T f = p.acc[a * n + k];
                    ph[a] = p.mom[a * n + k] - la.sub_k2 * f;
                    phd[a] = pdot[a * n + k] - la.sub_k2 * fdot[a * n + k] - ck2 * la.cell * f;
                }
                margin = min(la.sub_dr * max(max(fabs(ph[0]), fabs(ph[1])), fabs(ph[2])), nmf);
            }
            const int mz0 = max((int)floor(cnear / nmf), 0), mz1 = (int)floor(cfar / nmf);
            for (int nz = mz0; nz <= mz1; ++nz) {
                const T rz_hi = min(T(nz + 1) * nmf, cfar) + margin;
                const T rmax = tmax * rz_hi / la.inv_dtheta + margin;
                const int mx0 = (int)floor((-rmax + half) / nmf) - 1;
                const int mx1 = (int)floor((rmax + half) / nmf);
                for (int nx = mx0; nx <= mx1; ++nx)
                    for (int ny = mx0; ny <= mx1; ++ny) {
                        const int sym = la.rot ? vjp_replica_symmetry(nx, ny, nz, la.rot_seed) : 0;
                        T ui[3], ti[3], pi[3], qi[3];
#pragma unroll
                        for (int j = 0; j < 3; ++j) {
                            const int ax = vjp_sym_axis(sym, j);
                            const T c = ax == 0 ? u[0] : (ax == 1 ? u[1] : u[2]);
                            const T v = ax == 0 ? xb[0] : (ax == 1 ? xb[1] : xb[2]);
                            const T q = ax == 0 ? ph[0] : (ax == 1 ? ph[1] : ph[2]);
                            const T qd = ax == 0 ? phd[0] : (ax == 1 ? phd[1] : phd[2]);
                            const bool fl = (sym >> j) & 1;
                            ui[j] = fl ? nmf - c : c;
                            ti[j] = fl ? -v : v;
                            pi[j] = fl ? -q : q;
                            qi[j] = fl ? -qd : qd;
                        }
                        T rx = ui[0] + T(nx) * nmf - half, ry = ui[1] + T(ny) * nmf - half;
                        T rz = ui[2] + T(nz) * nmf;
                        int cr = cz;
                        T fr = fz;
                        if (sym) split_cell(ui[2], cr, fr);
                        if (!depth_in_shell(cr, fr, zbound<T>(la.cnear_d, nz, g.nm),
                                            zbound<T>(la.cfar_d, nz, g.nm)) ||
                            !(rz > T(0)))
                            continue;
                        if (la.sub) {
                            const T chi_e = rz * la.cell;
                            T de, dd;
                            tab_interp(la.dtab, la, chi_e, de, dd);
                            const T dr = (de - la.d_end) * la.sub_scale;
                            const T ddr = dd * la.sub_scale;  // per Mpc/h
                            const T ddr_dom = (lv.ddom_at(chi_e) - lv.dd_end_dom) * la.sub_scale +
                                              (de - la.d_end) * lv.dscale_dom;
                            const T zd = ti[2];
#pragma unroll
                            for (int j = 0; j < 3; ++j)
                                ti[j] += (ddr * zd + om_dot * ddr_dom) * pi[j] * la.cell + dr * qi[j];
                            rx += dr * pi[0];
                            ry += dr * pi[1];
                            rz += dr * pi[2];
                            if (!(rz > T(0))) continue;
                        }
                        const T chi = rz * la.cell;
                        if (chi >= chi_max_src) continue;
                        T a, dadchi;
                        a_interp(la, chi, a, dadchi);
                        lens_jvp_image(la, lv, kdot, npix2, rx, ry, rz, chi, a, dadchi,
                                       lv.dadom_at(chi), hp, dth, ti[0], ti[1], ti[2], om_dot);
                    }
            }
        } else {
            const int nz0 = (int)floor((cnear - u[2]) / nmf);
            const int nz1 = (int)floor((cfar - u[2]) / nmf) + 1;
            for (int nz = nz0; nz <= nz1; ++nz) {
                const T rz = u[2] + T(nz) * nmf;
                if (!depth_in_shell(cz, fz, zbound<T>(la.cnear_d, nz, g.nm),
                                    zbound<T>(la.cfar_d, nz, g.nm)) ||
                    !(rz > T(0)))
                    continue;
                const T chi = rz * la.cell;
                if (chi >= chi_max_src) continue;
                const T rmax = tmax * rz / la.inv_dtheta;
                const int nx0 = (int)floor((-rmax - u[0] + half) / nmf);
                const int nx1 = (int)floor((rmax - u[0] + half) / nmf) + 1;
                const int ny0 = (int)floor((-rmax - u[1] + half) / nmf);
                const int ny1 = (int)floor((rmax - u[1] + half) / nmf) + 1;
                T a, dadchi;
                a_interp(la, chi, a, dadchi);
                const T dadom = lv.dadom_at(chi);
                for (int nx = nx0; nx <= nx1; ++nx)
                    for (int ny = ny0; ny <= ny1; ++ny)
                        lens_jvp_image(la, lv, kdot, npix2, u[0] + T(nx) * nmf - half,
                                       u[1] + T(ny) * nmf - half, rz, chi, a, dadchi, dadom, hp,
                                       dth, xb[0], xb[1], xb[2], om_dot);
            }
        }
    }
}

// kdot[s] += v[s] on every pixel (the shell's mean term)
template <class T>
__global__ void k_map_add(T* kdot, long npix2, int nsrc, MapAdd<T> mv) {
    const long total = npix2 * nsrc;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x)
        kdot[i] += mv.v[i / npix2];
}

// ---------------------------------------------------------------------------
template <class T>
void launch_fvjp_readout(Parts<T> p, SortBufs s, Geo g, const T* f0, const T* f1, const T* f2,
                         const T* xbar_in, const T* pbar_in, T H, T ckick, T* xbc, T* fbc,
                         double* dots, uint32_t* fmax_bits, hipStream_t st) {
    int ntiles = g.nt * g.nt * g.nt;
    hipLaunchKernelGGL(k_fvjp_readout<T>, dim3(ntiles), dim3(AB), 0, st, p, s, g, f0, f1, f2,
                       xbar_in, pbar_in, H, ckick, xbc, fbc, dots, fmax_bits);
}

template <class T>
void launch_fvjp_paintgrad(Parts<T> p, SortBufs s, Geo g, const T* rhobar, T mass, const T* xbc,
                           T H, int mode, T dr, T k2, T d0, T gp0, T* xbar_out, const T* pbar_in,
                           T* pbar_out, const T* phbar, T* sb0, T* sb1, T* sb2, double* dots,
                           hipStream_t st) {
    int ntiles = g.nt * g.nt * g.nt;
    hipLaunchKernelGGL(k_fvjp_paintgrad<T>, dim3(ntiles), dim3(AB), 0, st, p, s, g, rhobar, mass,
                       xbc, H, mode, dr, k2, d0, gp0, xbar_out, pbar_in, pbar_out, phbar, sb0, sb1,
                       sb2, dots);
}

template <class T>
void launch_dot3(const T* a0, const T* a1, const T* a2, const T* b0, const T* b1, const T* b2,
                 long n, double* dst, hipStream_t st) {
    long blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_dot3<T>, dim3(blocks), dim3(256), 0, st, a0, a1, a2, b0, b1, b2, n, dst);
}

template <class T>
void launch_dot_sorted_lattice(Parts<T> p, Geo g, const T* sorted, const T* l0, const T* l1,
                               const T* l2, double* dst, hipStream_t st) {
    long blocks = (g.npart + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_dot_sorted_lattice<T>, dim3(blocks), dim3(256), 0, st, p, g, sorted, l0, l1,
                       l2, dst);
}

template <class T>
void launch_sorted_to_lattice(Parts<T> p, Geo g, const T* sorted, T* l0, T* l1, T* l2,
                              hipStream_t st) {
    long blocks = (g.npart + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_sorted_to_lattice<T>, dim3(blocks), dim3(256), 0, st, p, g, sorted, l0, l1, l2);
}

template <class T>
void launch_map_sums(const T* kbar, int npix, int nsrc, double* dst, hipStream_t st) {
    long npix2 = (long)npix * npix;
    long blocks = (npix2 + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(k_map_sums<T>, dim3(blocks), dim3(256), 0, st, kbar, npix2, nsrc, dst);
}

template <class T>
void launch_lens_vjp(Parts<T> p, Geo g, const LensArgs<T>& la, const LensVjpArgs<T>& lv,
                     const T* kbar, T* xbar, double* dots, hipStream_t st) {
    long blocks = (g.npart + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_lens_vjp<T>, dim3(blocks), dim3(256), 0, st, p, g, la, lv, kbar, xbar, dots);
}

static long grid_of(long n, long cap) {
    long blocks = (n + 255) / 256;
    return blocks > cap ? cap : (blocks < 1 ? 1 : blocks);
}

template <class T>
void launch_lin(T* y, const T* x, T a, T b, long n, hipStream_t st) {
    hipLaunchKernelGGL(k_lin<T>, dim3(grid_of(n, 16384)), dim3(256), 0, st, y, x, a, b, n);
}

template <class T>
void launch_ic_tangent(const T* t0, const T* t1, const T* t2, const T* s0, const T* s1,
                       const T* s2, T* xd, T* pd, T D, T gp, T cD, T cgp, T H, long n,
                       hipStream_t st) {
    hipLaunchKernelGGL(k_ic_tangent<T>, dim3(grid_of(n, 16384)), dim3(256), 0, st, t0, t1, t2, s0,
                       s1, s2, xd, pd, D, gp, cD, cgp, H, n);
}

template <class T>
void launch_lattice_to_sorted(Parts<T> p, Geo g, const T* lat, T* sorted, hipStream_t st) {
    hipLaunchKernelGGL(k_lattice_to_sorted<T>, dim3(grid_of(g.npart, 16384)), dim3(256), 0, st, p, g,
                       lat, sorted);
}

template <class T>
void launch_jvp_pre(Parts<T> p, Geo g, T* xdot, T* pdot, const T* fdot, T H, T k1, T dr, T ck1,
                    T cdr, hipStream_t st) {
    hipLaunchKernelGGL(k_jvp_pre<T>, dim3(grid_of(3 * g.npart, 16384)), dim3(256), 0, st, p, g,
                       xdot, pdot, fdot, H, k1, dr, ck1, cdr);
}

template <class T>
void launch_fjvp_gather(Parts<T> p, SortBufs s, Geo g, const T* f0, const T* f1, const T* f2,
                        const T* xdot, T invH, T mass, T* fbc, uint32_t* vmax_bits,
                        hipStream_t st) {
    int ntiles = g.nt * g.nt * g.nt;
    hipLaunchKernelGGL(k_fjvp_gather<T>, dim3(ntiles), dim3(AB), 0, st, p, s, g, f0, f1, f2, xdot,
                       invH, mass, fbc, vmax_bits);
}

template <class T>
void launch_fjvp_readout_kick(Parts<T> p, SortBufs s, Geo g, const T* m0, const T* m1, const T* m2,
                              const T* fbc, T H, T k2, T ck2, T* pdot, T* fdot, hipStream_t st) {
    int ntiles = g.nt * g.nt * g.nt;
    hipLaunchKernelGGL(k_fjvp_readout_kick<T>, dim3(ntiles), dim3(AB), 0, st, p, s, g, m0, m1, m2,
                       fbc, H, k2, ck2, pdot, fdot);
}

template <class T>
void launch_lens_jvp(Parts<T> p, Geo g, const LensArgs<T>& la, const LensVjpArgs<T>& lv,
                     const T* xdot, const T* pdot, const T* fdot, T ck2, T om_dot, T* kdot,
                     hipStream_t st) {
    hipLaunchKernelGGL(k_lens_jvp<T>, dim3(grid_of(g.npart, 16384)), dim3(256), 0, st, p, g, la,
                       lv, xdot, pdot, fdot, ck2, om_dot, kdot);
}

template <class T>
void launch_map_add(T* kdot, int npix, int nsrc, const MapAdd<T>& mv, hipStream_t st) {
    const long npix2 = (long)npix * npix;
    hipLaunchKernelGGL(k_map_add<T>, dim3(grid_of(npix2 * nsrc, 4096)), dim3(256), 0, st, kdot,
                       npix2, nsrc, mv);
}

__global__ void k_cosmo_acc(const double* dots, double* acc, CosmoCoef c) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double a0 = 0.0, a1 = 0.0;
    for (int i = 0; i < c.n; ++i) {
        a0 += c.c0[i] * dots[c.idx[i]];
        a1 += c.c1[i] * dots[c.idx[i]];
    }
    acc[0] += a0;
    acc[1] += a1;
}

void launch_cosmo_acc(const double* dots, double* acc, const CosmoCoef& c, hipStream_t st) {
    hipLaunchKernelGGL(k_cosmo_acc, dim3(1), dim3(64), 0, st, dots, acc, c);
}

#define ML_INST_JVP(T)                                                                               \
    template void launch_lin<T>(T*, const T*, T, T, long, hipStream_t);                              \
    template void launch_ic_tangent<T>(const T*, const T*, const T*, const T*, const T*, const T*,   \
                                       T*, T*, T, T, T, T, T, long, hipStream_t);                    \
    template void launch_lattice_to_sorted<T>(Parts<T>, Geo, const T*, T*, hipStream_t);             \
    template void launch_jvp_pre<T>(Parts<T>, Geo, T*, T*, const T*, T, T, T, T, T, hipStream_t);   \
    template void launch_fjvp_gather<T>(Parts<T>, SortBufs, Geo, const T*, const T*, const T*,       \
                                        const T*, T, T, T*, uint32_t*, hipStream_t);                 \
    template void launch_fjvp_readout_kick<T>(Parts<T>, SortBufs, Geo, const T*, const T*, const T*, \
                                              const T*, T, T, T, T*, T*, hipStream_t);               \
    template void launch_lens_jvp<T>(Parts<T>, Geo, const LensArgs<T>&, const LensVjpArgs<T>&,       \
                                     const T*, const T*, const T*, T, T, T*, hipStream_t);           \
    template void launch_map_add<T>(T*, int, int, const MapAdd<T>&, hipStream_t);
ML_INST_JVP(float)
ML_INST_JVP(double)

#define ML_INST(T)                                                                                   \
    template void launch_fvjp_readout<T>(Parts<T>, SortBufs, Geo, const T*, const T*, const T*,      \
                                         const T*, const T*, T, T, T*, T*, double*, uint32_t*,       \
                                         hipStream_t);                                               \
    template void launch_fvjp_paintgrad<T>(Parts<T>, SortBufs, Geo, const T*, T, const T*, T, int,   \
                                           T, T, T, T, T*, const T*, T*, const T*, T*, T*, T*,       \
                                           double*, hipStream_t);                                    \
    template void launch_dot3<T>(const T*, const T*, const T*, const T*, const T*, const T*, long,   \
                                 double*, hipStream_t);                                              \
    template void launch_map_sums<T>(const T*, int, int, double*, hipStream_t);                      \
    template void launch_dot_sorted_lattice<T>(Parts<T>, Geo, const T*, const T*, const T*, const T*, \
                                               double*, hipStream_t);                                \
    template void launch_sorted_to_lattice<T>(Parts<T>, Geo, const T*, T*, T*, T*, hipStream_t);     \
    template void launch_lens_vjp<T>(Parts<T>, Geo, const LensArgs<T>&, const LensVjpArgs<T>&,       \
                                     const T*, T*, double*, hipStream_t);
ML_INST(float)
ML_INST(double)

}  // namespace ml
