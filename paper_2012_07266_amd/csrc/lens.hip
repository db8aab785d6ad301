// Born lightcone projection on gfx950.
//
// The convergence of a source plane at comoving distance chi_s is the
// integral of (3/2) Om (H0/c)^2 q(chi) delta / a along the line of sight with
// q = chi (chi_s - chi) / chi_s (convergence equation of the paper's notation
// section).  With the particles of one PM step standing in for the density
// of its distance shell, every particle image r = x + n L - O (observer O at
// (L/2, L/2, 0), line of sight along axis 2, chi = r_2, theta = r_perp/chi)
// adds  wbase (chi_s - chi) / (chi_s chi a(chi))  to the map, bilinearly, and
// the shell's mean term is added to every pixel in the same pass.
#include "particles.h"
#include "batch.h"

namespace ml {

// Cubic Hermite interpolation of a table [ntab][2] of values and exact
// slopes on the grid chi_k = k dchi.
template <class T>
__device__ __forceinline__ T chi_table(const T* tab, const LensArgs<T>& la, T chi) {
    T xk = chi / la.dchi;
    int k = (int)floor(xk);
    k = min(max(k, 0), la.ntab - 2);
    T s = xk - T(k);
    T a0 = tab[2 * k], d0 = tab[2 * k + 1] * la.dchi;
    T a1 = tab[2 * k + 2], d1 = tab[2 * k + 3] * la.dchi;
    T s2 = s * s, s3 = s2 * s;
    return (T(2) * s3 - T(3) * s2 + T(1)) * a0 + (s3 - T(2) * s2 + s) * d0 +
           (T(3) * s2 - T(2) * s3) * a1 + (s3 - s2) * d1;
}

template <class T>
__device__ __forceinline__ T a_of_chi(const LensArgs<T>& la, T chi) {
    return chi_table(la.atab, la, chi);
}

// chi_table from a copy of entries k_lo .. k_hi held at w[2 (k - k_lo)]
template <class T>
__device__ __forceinline__ T chi_window(const T* w, int k_lo, int k_hi, const LensArgs<T>& la,
                                        T chi) {
    T xk = chi / la.dchi;
    int k = (int)floor(xk);
    k = min(max(k, 0), la.ntab - 2);
    k = min(max(k, k_lo), k_hi - 1);
    T s = xk - T(k);
    const T* e = w + 2 * (k - k_lo);
    T a0 = e[0], d0 = e[1] * la.dchi;
    T a1 = e[2], d1 = e[3] * la.dchi;
    T s2 = s * s, s3 = s2 * s;
    return (T(2) * s3 - T(3) * s2 + T(1)) * a0 + (s3 - T(2) * s2 + s) * d0 +
           (T(3) * s2 - T(2) * s3) * a1 + (s3 - s2) * d1;
}

// ---------------------------------------------------------------------------
// Replica rotation: the 64-bit finalizer of SplitMix64 (Steele, Lea and
// Flood, 2014) hashes a replica's offsets and the seed to one of the 48 cube
// symmetries.  Symmetry s takes axis permutation s / 8 of the six in
// lexicographic order and reflects image axis j when bit j of s % 8 is set;
// image axis j is box axis perm(j), x -> Nm - x when reflected.
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ int replica_symmetry(int nx, int ny, int nz, unsigned long long seed) {
    const unsigned long long u = ((unsigned long long)(nx + (1 << 20)) << 42) |
                                 ((unsigned long long)(ny + (1 << 20)) << 21) |
                                 (unsigned long long)(nz + (1 << 20));
    return (int)(mix64(seed ^ mix64(u)) % 48ull);
}

// perm(j) of symmetry s: the permutation's first entry is (s / 8) / 2, the
// other two follow in increasing order, swapped when (s / 8) is odd
__device__ __forceinline__ int sym_axis(int s, int j) {
    const int p = s >> 3, f = p >> 1;
    const int r0 = f == 0 ? 1 : 0, r1 = f == 2 ? 1 : 2;
    return j == 0 ? f : (j == 1 ? ((p & 1) ? r1 : r0) : ((p & 1) ? r0 : r1));
}

// v in the image frame: component j is v[perm(j)], reflected (about `refl`:
// Nm for positions, 0 with a sign flip for vectors) when flip j is set
template <class T>
__device__ __forceinline__ void sym_apply(int s, T (&v)[3], T refl, bool vec) {
    const T v0 = v[0], v1 = v[1], v2 = v[2];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const int a = sym_axis(s, j);
        T c = a == 0 ? v0 : (a == 1 ? v1 : v2);
        if ((s >> j) & 1) c = vec ? -c : refl - c;
        v[j] = c;
    }
}

// ---------------------------------------------------------------------------
// Region-driven projection: a workgroup owns a RS x RS pixel region of every
// map.  For each box replica it bounds the part of the shell that projects
// into the region (with a one-pixel margin for bilinear spill), visits the
// particle tiles inside that bound (tile-sorted particles, so each (tx, ty)
// column over a z range is one contiguous index range), and accumulates the
// region in LDS.  float: 64-bit fixed point with 40 fractional bits (exact,
// order-independent sums at full integer-atomic rate); an image weight of
// 2^22 or more (a particle within ~1e-5 Mpc/h of the observer) goes to the
// map directly with a float atomic.  double: float64 LDS atomics.  Each
// pixel is then written by exactly one workgroup, together with the shell's
// mean term.
// ---------------------------------------------------------------------------
template <class T> struct LensAcc;
template <> struct LensAcc<float> {
    using S = unsigned long long;
    static constexpr float LIM = 4194304.0f;  // 2^22
    static __device__ __forceinline__ S enc(float w) {
        return (S)__float2ull_rn(w * 1099511627776.0f);  // 2^40
    }
    static __device__ __forceinline__ float dec(S v) {
        return (float)((double)v * (1.0 / 1099511627776.0));
    }
    static __device__ __forceinline__ double dec_d(S v) { return (double)v * (1.0 / 1099511627776.0); }
};
template <> struct LensAcc<double> {
    using S = double;
    static constexpr double LIM = 1e300;
    static __device__ __forceinline__ S enc(double w) { return w; }
    static __device__ __forceinline__ double dec(S v) { return v; }
    static __device__ __forceinline__ double dec_d(S v) { return v; }
};

// The bilinear splat of weight w at pixel coordinates (t0, t1) into the
// region's accumulator, a corner weight at or above the fixed-point limit
// (or every corner, global_only) going to the map kmap with a float atomic.
template <class T>
__device__ __forceinline__ void splat_region(typename LensAcc<T>::S* acc, int rs, int p0x, int p0y,
                                             int npix, T* kmap, T t0, T t1, T w,
                                             bool global_only = false) {
    using A = LensAcc<T>;
    T fl0 = floor(t0), fl1 = floor(t1);
    int j0 = (int)fl0, j1 = (int)fl1;
    T f0 = t0 - fl0, f1 = t1 - fl1;
    T wa[2] = {T(1) - f0, f0}, wb[2] = {T(1) - f1, f1};
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        int r = j0 + a;
        if (r < p0x || r >= p0x + rs || r >= npix) continue;
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            int c = j1 + b;
            if (c < p0y || c >= p0y + rs || c >= npix) continue;
            T v = w * wa[a] * wb[b];
            if (!global_only && v < T(A::LIM)) atomicAdd(&acc[(r - p0x) * rs + (c - p0y)], A::enc(v));
            else unsafeAtomicAdd(&kmap[(long)r * npix + c], v);
        }
    }
}

// Depth range [zmin, zmax] (cells from the observer) over which images of a
// tile column whose transverse coordinate spans [Xa, Xa + TILE) can fall in
// the angular window [alo, ahi] (X / Z in the window, with `margin` cells of
// slack); false when empty.  The window of a map region is a thin slanted
// pencil, so a column meets it over one depth interval.
template <class T>
__device__ __forceinline__ bool column_depths(T alo, T ahi, T Xa, T margin, T& zmin, T& zmax) {
    const T U = Xa + T(TILE) + margin, L = Xa - margin;
    // alo Z <= U
    if (alo > T(0)) zmax = min(zmax, U / alo);
    else if (U < T(0)) {
        if (alo < T(0)) zmin = max(zmin, U / alo);
        else return false;
    }
    // ahi Z >= L
    if (ahi < T(0)) {
        if (L < T(0)) zmax = min(zmax, L / ahi);
        else return false;
    } else if (L > T(0)) {
        if (ahi > T(0)) zmin = max(zmin, L / ahi);
        else return false;
    }
    return zmin <= zmax;
}

constexpr int LU = 4;   // particles per thread in flight
constexpr int LQ = 128;  // entries of a wave's image queue (63 waiting + 64 new at most)

// LDS bytes of the image queues of an LG-thread workgroup (float only)
template <class T> constexpr size_t lens_queue_bytes(int lg) {
    return sizeof(T) == 4 ? (size_t)(lg / 64) * 3 * LQ * sizeof(T) : 0;
}

// LG threads per workgroup: 256 for 32 x 32-pixel regions, 1024 for 64 x 64
// (one workgroup per CU then holds the LDS, so it brings 16 waves)
// DEC: the maps of the sources beyond the shell come from the shared
// accumulators A and B (la.dec); else one accumulator per source.
template <class T, int LG, bool EXT, bool DEC>
__device__ __forceinline__ void lens_gather_body(Parts<T> p, SortBufs sb, Geo g, LensArgs<T> la,
                                                    MapAdd<T> mean, T* kappa) {
    using A = LensAcc<T>;
    using S = typename A::S;
    constexpr int LUT = sizeof(T) == 4 ? LU : LU / 2;  // registers of double
    constexpr bool COMPACT = sizeof(T) == 4;
    extern __shared__ unsigned char smem[];
    S* acc = reinterpret_cast<S*>(smem);
    const int rs = la.rs;
    const int nreg = (la.npix + rs - 1) / rs;
    // renumber workgroups so each of the 8 XCDs (round-robin dispatch) walks a
    // contiguous band of regions: neighbouring regions read the same particle
    // tiles, which then stay in that XCD's L2
    int b = blockIdx.x;
    if (gridDim.x % 8 == 0) b = (b % 8) * (gridDim.x / 8) + b / 8;
    const int rx = b / nreg, ry = b % nreg;
    const int p0x = rx * rs, p0y = ry * rs;
    const int tid = threadIdx.x;
    const int rs2 = rs * rs;
    const int ncell = (DEC ? la.nacc : la.nsrc) * rs2;
    for (int i = tid; i < ncell; i += LG) acc[i] = S(0);
    // sub-evolution: the part of the D(a(chi)) table that end-of-step
    // depths in the shell can reach (one entry of margin below, two above)
    // is copied after the accumulator when it fits in la.dwin entries; the
    // clamp to the window never moves an index of such a depth, so the
    // values are those of the table itself
    T* dw = reinterpret_cast<T*>(acc + ncell);
    int d_lo = 0, d_hi = 0;
    bool d_lds = false;
    if (EXT && la.sub) {
        d_lo = min(max((int)floor(la.chi_near / la.dchi) - 1, 0), la.ntab - 2);
        d_hi = min(max((int)floor(la.chi_far / la.dchi) + 2, d_lo + 1), la.ntab - 1);
        d_lds = d_hi - d_lo + 1 <= la.dwin;
        if (d_lds)
            for (int i = tid; i < 2 * (d_hi - d_lo + 1); i += LG) dw[i] = la.dtab[2 * d_lo + i];
    }
    __syncthreads();

    const long n = g.npart;
    const int nm = g.nm, nt = g.nt;
    const T nmf = T(nm), half = T(0.5) * nmf;
    const T hp = T(0.5) * T(la.npix) - T(0.5);
    const T cnear = la.chi_near / la.cell, cfar = la.chi_far / la.cell;  // cells
    T chi_max_src = la.chi_src[0];
    for (int s = 1; s < la.nsrc; ++s) chi_max_src = max(chi_max_src, la.chi_src[s]);
    const T cmax = min(cfar, chi_max_src / la.cell);
    const T dth = T(1) / la.inv_dtheta;
    // angular window of images touching the region: t in [p0 - 1, p0 + rs)
    const T a0lo = (T(p0x - 1) - hp) * dth, a0hi = (T(p0x + rs) - hp) * dth;
    const T a1lo = (T(p0y - 1) - hp) * dth, a1hi = (T(p0y + rs) - hp) * dth;
    // cells of slack on every bound; with sub-evolution also the largest
    // move of an image (the step's drift factor times max |p_h|), with a
    // shift (PGD) its largest size; each capped at one box so that the
    // replica ranges stay bounded whatever the inputs
    T margin = T(1);
    // a shifted image can leave its replica's box by up to the shift (it is
    // added to the wrapped position, not wrapped again)
    T zclip = T(0);
    if constexpr (EXT) {
        if (la.sub) margin += min(la.sub_dr * (T)__uint_as_float(*la.pmax_bits), nmf);
        if (la.shift) {
            zclip = min(fabs(la.shift_scale) * (T)__uint_as_float(*la.shift_bits), nmf);
            margin += zclip;
        }
    }
    const int npix2 = la.npix * la.npix;
    // an accepted image: its weight for every source behind it, bilinearly
    // into the region (the shared accumulators A and B for the sources
    // beyond the shell, unless the weight is near the fixed-point limit:
    // then per source, as for the sources of their own)
    auto deposit = [&](T t0, T t1, T chi) {
        T base_w = la.wbase / (chi * a_of_chi(la, chi));
        if constexpr (!DEC) {
            for (int s = 0; s < la.nsrc; ++s) {
                T cs = la.chi_src[s];
                if (chi < cs)
                    splat_region<T>(acc + s * rs2, rs, p0x, p0y, la.npix, kappa + (long)s * npix2,
                                    t0, t1, base_w * (cs - chi) / cs);
            }
            return;
        }
        if (base_w < T(0.5) * T(A::LIM)) {
            // every corner weight is below the limit: the map argument is
            // never written
            splat_region<T>(acc, rs, p0x, p0y, la.npix, kappa, t0, t1, base_w);
            splat_region<T>(acc + rs2, rs, p0x, p0y, la.npix, kappa, t0, t1,
                            base_w * chi * la.inv_chi_ref);
        } else {
            for (int s = 0; s < la.nsrc; ++s) {
                if (la.slot[s] != -1) continue;
                T cs = la.chi_src[s];
                splat_region<T>(acc, rs, p0x, p0y, la.npix, kappa + (long)s * npix2, t0, t1,
                                base_w * (cs - chi) / cs, true);
            }
        }
        for (int d = 0; d < la.ndirect; ++d) {
            const int s = la.direct_src[d];
            T cs = la.chi_src[s];
            if (chi < cs)
                splat_region<T>(acc + (2 + d) * rs2, rs, p0x, p0y, la.npix,
                                kappa + (long)s * npix2, t0, t1, base_w * (cs - chi) / cs);
        }
    };
    // float: a wave's accepted images wait in its own LDS queue (after the
    // accumulator and the D window) until 64 of them fill every lane, so
    // the weights and splats run on full waves, not on the few lanes of each
    // visit that land in the region.  The queue count is wave-uniform, and
    // a wave's LDS accesses complete in order, so no barrier is needed.
    const int dwin = (EXT && la.sub) ? la.dwin : 0;
    T* q = reinterpret_cast<T*>(smem + (size_t)ncell * sizeof(S) + (size_t)dwin * 2 * sizeof(T)) +
           (tid >> 6) * 3 * LQ;
    const int lane = tid & 63;
    int qn = 0;
    auto queue_push = [&](bool ok, T t0, T t1, T chi) {
        const unsigned long long m = __ballot(ok);
        if (!m) return;
        if (ok) {
            const int pos = qn + (int)__builtin_amdgcn_mbcnt_hi(
                                     (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
            q[pos] = t0;
            q[LQ + pos] = t1;
            q[2 * LQ + pos] = chi;
        }
        qn += __popcll(m);
        if (qn >= 64) {
            issue_fence();  // the stores above stay before the loads
            qn -= 64;
            const int e = qn + lane;
            deposit(q[e], q[LQ + e], q[2 * LQ + e]);
            issue_fence();  // and these loads before the next stores
        }
    };

    // the first and last sort block, within a tile column, of the tile at
    // depth z (cells; a column's blocks run along axis 2 a tile at a time)
    auto first_block_at = [](T z) { return (int)floor(z / T(TILE)) * BPT; };
    auto last_block_at = [](T z) { return (int)floor(z / T(TILE)) * BPT + BPT - 1; };
    int nz0 = (int)floor(cnear / nmf) - 1;
    if (nz0 < 0) nz0 = 0;
    const int nz1 = (int)floor(cmax / nmf) + (zclip > T(0) ? 1 : 0);
    for (int nz = nz0; nz <= nz1; ++nz) {
        T zlo = max(cnear - T(nz) * nmf, -zclip), zhi = min(cmax - T(nz) * nmf, nmf + zclip);
        if (!(zlo < zhi)) continue;
        T ca = zlo + T(nz) * nmf, cb = zhi + T(nz) * nmf;  // depth range, cells
        const ZBound<T> zb_near = zbound<T>(la.cnear_d, nz, nm), zb_far = zbound<T>(la.cfar_d, nz, nm);
        T x0lo = min(a0lo * ca, a0lo * cb) - margin, x0hi = max(a0hi * ca, a0hi * cb) + margin;
        T x1lo = min(a1lo * ca, a1lo * cb) - margin, x1hi = max(a1hi * ca, a1hi * cb) + margin;
        // sort blocks of the tiles (TILE cells deep) along axis 2 that the
        // replica's depth range can reach
        int tz0 = max(first_block_at(zlo - margin), 0);
        int tz1 = min(last_block_at(zhi + margin), g.ncb - 1);
        int nx0 = (int)floor((x0lo + half) / nmf), nx1 = (int)floor((x0hi + half) / nmf);
        int ny0 = (int)floor((x1lo + half) / nmf), ny1 = (int)floor((x1hi + half) / nmf);
        for (int nx = nx0; nx <= nx1; ++nx) {
            T bxlo = x0lo + half - T(nx) * nmf, bxhi = x0hi + half - T(nx) * nmf;  // box x, cells
            for (int ny = ny0; ny <= ny1; ++ny) {
                T bylo = x1lo + half - T(ny) * nmf, byhi = x1hi + half - T(ny) * nmf;
                int sym = 0;
                if constexpr (EXT) {
                    if (la.rot) sym = replica_symmetry(nx, ny, nz, la.rot_seed);
                }
                // the image-frame box [b*lo, b*hi] in box axes: the tiles and
                // sort blocks to visit (a rotated replica is culled by this
                // box alone; an unrotated one also per column below)
                T lo3[3] = {bxlo, bylo, zlo - margin}, hi3[3] = {bxhi, byhi, zhi + margin};
                if (sym) {
                    const T l0 = lo3[0], l1 = lo3[1], l2 = lo3[2];
                    const T h0 = hi3[0], h1 = hi3[1], h2 = hi3[2];
#pragma unroll
                    for (int j = 0; j < 3; ++j) {  // image axis j -> box axis sym_axis(sym, j)
                        const T lj = j == 0 ? l0 : (j == 1 ? l1 : l2);
                        const T hj = j == 0 ? h0 : (j == 1 ? h1 : h2);
                        const bool fl = (sym >> j) & 1;
                        const T a = fl ? nmf - hj : lj, b = fl ? nmf - lj : hj;
                        const int ax = sym_axis(sym, j);
#pragma unroll
                        for (int q = 0; q < 3; ++q)
                            if (q == ax) {
                                lo3[q] = a;
                                hi3[q] = b;
                            }
                    }
                }
                const int tx0 = max((int)floor(lo3[0] / T(TILE)), 0);
                const int tx1 = min((int)floor(hi3[0] / T(TILE)), nt - 1);
                const int ty0 = max((int)floor(lo3[1] / T(TILE)), 0);
                const int ty1 = min((int)floor(hi3[1] / T(TILE)), nt - 1);
                const int kza = sym ? max(first_block_at(lo3[2]), 0) : tz0;
                const int kzb = sym ? min(last_block_at(hi3[2]), g.ncb - 1) : tz1;
                for (int tx = tx0; tx <= tx1; ++tx)
                    for (int ty = ty0; ty <= ty1; ++ty) {
                        int tza = kza, tzb = kzb;
                        if (!sym) {
                            // only the tiles of this column that the region's
                            // pencil crosses
                            T zmin = ca - margin, zmax = cb + margin;
                            if (!column_depths(a0lo, a0hi, T(tx * TILE) + T(nx) * nmf - half,
                                               margin, zmin, zmax) ||
                                !column_depths(a1lo, a1hi, T(ty * TILE) + T(ny) * nmf - half,
                                               margin, zmin, zmax))
                                continue;
                            tza = max(tz0, first_block_at(zmin - T(nz) * nmf));
                            tzb = min(tz1, last_block_at(zmax - T(nz) * nmf));
                        }
                        if (tza > tzb) continue;
                        const int col = (tx * nt + ty) * g.ncb;
                        const uint32_t lo = sb.start[col + tza], hi = sb.start[col + tzb + 1];
                        for (uint32_t base = lo; base < hi; base += LG * LUT) {
                            uint32_t idv[LUT];
                            T dv[LUT][3], pv[EXT ? LUT : 1][3], sv[EXT ? LUT : 1][3];
#pragma unroll
                            for (int u = 0; u < LUT; ++u) {
                                uint32_t k = base + u * LG + tid;
                                if (k < hi) {
                                    idv[u] = p.id[k];
                                    dv[u][0] = p.disp[k];
                                    dv[u][1] = p.disp[n + k];
                                    dv[u][2] = p.disp[2 * n + k];
                                    if constexpr (EXT) {
                                        if (la.sub) {
#pragma unroll
                                            for (int a = 0; a < 3; ++a) {
                                                pv[u][a] = p.mom[a * n + k];
                                                if (la.sub_k2 != T(0))
                                                    pv[u][a] -= la.sub_k2 * p.acc[a * n + k];
                                            }
                                        }
                                        if (la.shift) {
#pragma unroll
                                            for (int a = 0; a < 3; ++a)
                                                sv[u][a] = la.shift[a * n + k];
                                        }
                                    }
                                }
                            }
                            // the particle's image in this replica: its pixel coordinates and
                            // distance when it falls in the shell and in the region's window
                            auto image = [&](int u, T& t0, T& t1, T& chi) -> bool {
                                int li[3];
                                lattice_of_l(idv[u], g.np, li);
                                T uu[3];
                                int cz = 0;
                                T fz = T(0);
#pragma unroll
                                for (int a = 0; a < 3; ++a) {
                                    T v = T(0.5) + dv[u][a];
                                    T fl = floor(v);
                                    int c = g.B * li[a] + (int)fl;
                                    if ((unsigned)c >= (unsigned)nm) c = pmod(c, nm);
                                    uu[a] = T(c) + (v - fl);
                                    if (a == 2) {
                                        cz = c;
                                        fz = v - fl;
                                    }
                                }
                                T pimg[3] = {T(0), T(0), T(0)};
                                if constexpr (EXT) {
                                    if (la.shift) {  // PGD: on the wrapped position
#pragma unroll
                                        for (int a = 0; a < 3; ++a)
                                            uu[a] += la.shift_scale * sv[u][a];
                                    }
                                    if (la.sub) {
#pragma unroll
                                        for (int a = 0; a < 3; ++a) pimg[a] = pv[u][a];
                                    }
                                    if (sym) {  // into the replica's frame
                                        sym_apply(sym, uu, nmf, false);
                                        sym_apply(sym, pimg, T(0), true);
                                    }
                                    if (sym || la.shift) split_cell(uu[2], cz, fz);
                                }
                                T rz = uu[2] + T(nz) * nmf;
                                if (!depth_in_shell(cz, fz, zb_near, zb_far) || !(rz > T(0))) return false;
                                if (EXT && la.sub) {
                                    // along the step's drift to a(chi) of the
                                    // end-of-step depth
                                    const T chi_e = rz * la.cell;
                                    const T dd = ((d_lds ? chi_window(dw, d_lo, d_hi, la, chi_e)
                                                         : chi_table(la.dtab, la, chi_e)) -
                                                  la.d_end) *
                                                 la.sub_scale;
                                    uu[0] += dd * pimg[0];
                                    uu[1] += dd * pimg[1];
                                    rz += dd * pimg[2];
                                    if (!(rz > T(0))) return false;
                                }
                                chi = rz * la.cell;
                                if (!(chi < chi_max_src)) return false;
                                T inv = la.inv_dtheta / rz;
                                t0 = (uu[0] + T(nx) * nmf - half) * inv + hp;
                                t1 = (uu[1] + T(ny) * nmf - half) * inv + hp;
                                if (!(t0 >= T(p0x - 1) && t0 < T(p0x + rs) && t0 > T(-1) &&
                                      t1 >= T(p0y - 1) && t1 < T(p0y + rs) && t1 > T(-1)))
                                    return false;
                                return true;
                            };
#pragma unroll
                            for (int u = 0; u < LUT; ++u) {
                                const uint32_t k = base + u * LG + tid;
                                T t0 = T(0), t1 = T(0), chi = T(0);
                                const bool ok = k < hi && image(u, t0, t1, chi);
                                if constexpr (COMPACT) {
                                    queue_push(ok, t0, t1, chi);
                                } else {
                                    if (ok) deposit(t0, t1, chi);
                                }
                            }
                        }
                    }
            }
        }
    }
    if (COMPACT && qn > 0) {  // the images left in the queue
        issue_fence();
        if (lane < qn) deposit(q[lane], q[LQ + lane], q[2 * LQ + lane]);
    }
    __syncthreads();
    for (int i = tid; i < la.nsrc * rs2; i += LG) {
        const int s = i / rs2, rc = i - s * rs2, r = rc / rs, c = rc % rs;
        int px = p0x + r, py = p0y + c;
        if (px < la.npix && py < la.npix) {
            long o = (long)s * npix2 + (long)px * la.npix + py;
            T v;
            if constexpr (DEC) {
                const int sl = la.slot[s];
                v = T(0);
                if (sl >= 0) v = A::dec(acc[sl * rs2 + rc]);
                else if (sl == -1)
                    v = (T)(A::dec_d(acc[rc]) - la.ratio[s] * A::dec_d(acc[rs2 + rc]));
            } else {
                v = A::dec(acc[i]);
            }
            kappa[o] += v + mean.v[s];
        }
    }
}

template <class T, int LG, bool EXT, bool DEC>
__global__ __launch_bounds__(LG) void k_lens_gather(Parts<T> p, SortBufs sb, Geo g, LensArgs<T> la,
                                                    MapAdd<T> mean, T* kappa) {
    lens_gather_body<T, LG, EXT, DEC>(p, sb, g, la, mean, kappa);
}
template <class T, int LG>
__global__ __launch_bounds__(LG) void k_lens_gather_b(const LensGatherArgs<T>* __restrict__ tab) {
    const LensGatherArgs<T> a = tab[blockIdx.y];
    if (!a.on) return;
    lens_gather_body<T, LG, false, false>(a.p, a.sb, a.g, a.la, a.mean, a.kappa);
}

// LDS bytes after the accumulator for the D(a(chi)) window of sub-evolution
constexpr size_t DWIN_BYTES = 16384;

template <class T, int LG, bool EXT, bool DEC>
static void launch_lens_gather_k(Parts<T> p, SortBufs sb, Geo g, const LensArgs<T>& la,
                                 const MapAdd<T>& mean, T* kappa, size_t lds, hipStream_t st) {
    constexpr size_t LDS_MAX = 163840;  // per workgroup on gfx950
    // above the default dynamic LDS limit: raised once per instantiation
    static bool raised = false;
    if (!raised) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_lens_gather<T, LG, EXT, DEC>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)LDS_MAX);
        raised = true;
    }
    const int nreg = (la.npix + la.rs - 1) / la.rs;
    hipLaunchKernelGGL((k_lens_gather<T, LG, EXT, DEC>), dim3(nreg * nreg), dim3(LG), lds, st, p,
                       sb, g, la, mean, kappa);
}

template <class T, bool EXT>
void launch_lens_gather_t(Parts<T> p, SortBufs sb, Geo g, LensArgs<T> la,
                          const MapAdd<T>& mean, T* kappa, hipStream_t st) {
    const int lg = la.rs >= 64 ? 1024 : 256;
    size_t lds = (size_t)(la.dec ? la.nacc : la.nsrc) * la.rs * la.rs *
                     sizeof(typename LensAcc<T>::S) +
                 lens_queue_bytes<T>(lg);
    constexpr size_t LDS_MAX = 163840;  // per workgroup on gfx950
    la.dwin = 0;
    if (EXT && la.sub && lds < LDS_MAX) {
        // as much of DWIN_BYTES as the accumulator and the queues leave
        const size_t w = std::min(DWIN_BYTES, LDS_MAX - lds) / (2 * sizeof(T));
        la.dwin = (int)w;
        lds += w * 2 * sizeof(T);
    }
    if (lg == 1024) {
        if (la.dec) launch_lens_gather_k<T, 1024, EXT, true>(p, sb, g, la, mean, kappa, lds, st);
        else launch_lens_gather_k<T, 1024, EXT, false>(p, sb, g, la, mean, kappa, lds, st);
    } else {
        if (la.dec) launch_lens_gather_k<T, 256, EXT, true>(p, sb, g, la, mean, kappa, lds, st);
        else launch_lens_gather_k<T, 256, EXT, false>(p, sb, g, la, mean, kappa, lds, st);
    }
}

// The plain projection over the slots of a batch (one shape: the map size,
// source count and region side of `shape` are every slot's).
// Raises the batched kernels' dynamic LDS limit (before any capture).
template <class T>
void prepare_lens_gather_batch() {
    constexpr size_t LDS_MAX = 163840;  // per workgroup on gfx950
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_lens_gather_b<T, 1024>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)LDS_MAX);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_lens_gather_b<T, 256>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)LDS_MAX);
}

template <class T>
void launch_lens_gather_batch(const LensGatherArgs<T>* tab, const LensArgs<T>& shape, int slots,
                              hipStream_t st) {
    const int nreg = (shape.npix + shape.rs - 1) / shape.rs;
    const size_t lds = (size_t)shape.nsrc * shape.rs * shape.rs * sizeof(typename LensAcc<T>::S) +
                       lens_queue_bytes<T>(shape.rs >= 64 ? 1024 : 256);
    if (shape.rs >= 64)
        hipLaunchKernelGGL((k_lens_gather_b<T, 1024>), dim3(nreg * nreg, slots), dim3(1024), lds, st,
                           tab);
    else
        hipLaunchKernelGGL((k_lens_gather_b<T, 256>), dim3(nreg * nreg, slots), dim3(256), lds, st,
                           tab);
}

// The plain projection is its own instantiation, free of the per-particle
// loads and moves of sub-evolution and of the PGD shift.
template <class T>
void launch_lens_gather(Parts<T> p, SortBufs sb, Geo g, const LensArgs<T>& la,
                        const MapAdd<T>& mean, T* kappa, hipStream_t st) {
    if (la.sub || la.shift || la.rot)
        launch_lens_gather_t<T, true>(p, sb, g, la, mean, kappa, st);
    else
        launch_lens_gather_t<T, false>(p, sb, g, la, mean, kappa, st);
}

// Largest |mom - k2 acc| over particles and axes, for the frustum margin of
// sub-evolution: a wave maximum, then one atomic per wave on the bits of a
// non-negative float (whose unsigned order is the float order), rounded up.
template <class T>
__global__ __launch_bounds__(256) void k_drift_momentum_max(Parts<T> p, long n3, T k2,
                                                            uint32_t* out) {
    // 16 bytes a load, RU loads in flight per thread
    constexpr int VW = 16 / (int)sizeof(T), RU = 4;
    using V = T __attribute__((ext_vector_type(16 / sizeof(T))));
    float m = 0.0f;
    const long nv = n3 / VW;  // whole vectors (the arrays are 256-byte aligned)
    for (long base = (long)blockIdx.x * 256 * RU; base < nv; base += (long)gridDim.x * 256 * RU) {
        V v[RU], f[RU];
#pragma unroll
        for (int r = 0; r < RU; ++r) {
            long i = base + r * 256 + threadIdx.x;
            i = i < nv ? i : nv - 1;   // a repeat, harmless for a maximum
            v[r] = reinterpret_cast<const V*>(p.mom)[i];
            if (k2 != T(0)) f[r] = reinterpret_cast<const V*>(p.acc)[i];
        }
#pragma unroll
        for (int r = 0; r < RU; ++r)
#pragma unroll
            for (int e = 0; e < VW; ++e) {
                T x = v[r][e];
                if (k2 != T(0)) x -= k2 * f[r][e];
                m = fmaxf(m, (float)fabs(x));
            }
    }
    for (long i = nv * VW + (long)blockIdx.x * 256 + threadIdx.x; i < n3;
         i += (long)gridDim.x * 256) {  // the tail
        T x = p.mom[i];
        if (k2 != T(0)) x -= k2 * p.acc[i];
        m = fmaxf(m, (float)fabs(x));
    }
    // workgroup maximum, then one atomic per workgroup (atomics on one
    // address serialize in its L2 channel)
    __shared__ float wmax[4];
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        m = fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3]));
        atomicMax(out, __float_as_uint(m * 1.00001f));
    }
}

template <class T>
void launch_drift_momentum_max(Parts<T> p, long n, T k2, uint32_t* out, hipStream_t st) {
    constexpr int VW = 16 / (int)sizeof(T);
    long blocks = (3 * n / VW + 256 * 4 - 1) / (256 * 4);
    if (blocks > 1024) blocks = 1024;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_drift_momentum_max<T>, dim3(blocks), dim3(256), 0, st, p, 3 * n, k2, out);
}

template void launch_drift_momentum_max<float>(Parts<float>, long, float, uint32_t*, hipStream_t);
template void launch_drift_momentum_max<double>(Parts<double>, long, double, uint32_t*,
                                                hipStream_t);

template void launch_lens_gather<float>(Parts<float>, SortBufs, Geo, const LensArgs<float>&,
                                        const MapAdd<float>&, float*, hipStream_t);
template void launch_lens_gather<double>(Parts<double>, SortBufs, Geo, const LensArgs<double>&,
                                         const MapAdd<double>&, double*, hipStream_t);


template void prepare_lens_gather_batch<float>();
template void prepare_lens_gather_batch<double>();
template void launch_lens_gather_batch<float>(const LensGatherArgs<float>*,
                                              const LensArgs<float>&, int, hipStream_t);
template void launch_lens_gather_batch<double>(const LensGatherArgs<double>*,
                                               const LensArgs<double>&, int, hipStream_t);

}  // namespace ml
