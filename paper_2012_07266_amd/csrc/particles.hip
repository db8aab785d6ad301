// Particle kernels of the PM step on gfx950: counting sort by 16^3-cell
// tile, LDS-tiled cloud-in-cell paint with a deterministic halo merge,
// LDS-staged CIC force readout fused with the kick, kick/drift fused with
// the sort histogram, and the conversions between the tile-sorted internal
// state and lattice-ordered positions/momenta.
//
// Mass assignment is cloud-in-cell: a particle at cell coordinate u
// (node m at u = m) gives weight (1 - t) to node floor(u) and t to node
// floor(u) + 1 along each axis, t = u - floor(u), nodes taken modulo Nm.
#include "particles.h"

namespace ml {

constexpr int PB = 256;  // threads per workgroup of the particle kernels

__device__ __forceinline__ void lattice_of(uint32_t id, int np, int& i0, int& i1, int& i2) {
    i2 = (int)(id % (uint32_t)np);
    uint32_t r = id / (uint32_t)np;
    i1 = (int)(r % (uint32_t)np);
    i0 = (int)(r / (uint32_t)np);
}

// Base cell (wrapped) and fraction along one axis from the lattice index and
// the displacement.  The integer part of the lattice point stays exact.
template <class T>
__device__ __forceinline__ void cell_of(int B, int i, T disp, int nm, int& c, T& t) {
    T v = T(0.5) + disp;
    T fl = floor(v);
    t = v - fl;
    c = pmod(B * i + (int)fl, nm);
}

template <class T>
__device__ __forceinline__ bool finite3(T a, T b, T c) {
    return isfinite(a) && isfinite(b) && isfinite(c) && fabs(a) < T(1e6) && fabs(b) < T(1e6) &&
           fabs(c) < T(1e6);
}

// ---------------------------------------------------------------------------
template <class T>
__global__ void k_fill(T* p, T v, long n) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        p[i] = v;
}

template <class T>
void launch_fill(T* p, T v, long n, hipStream_t st) {
    long blocks = (n + PB - 1) / PB;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_fill<T>, dim3(blocks), dim3(PB), 0, st, p, v, n);
}
void launch_fill_u32(uint32_t* p, uint32_t v, long n, hipStream_t st) { launch_fill<uint32_t>(p, v, n, st); }

template <class T>
__global__ void k_scale_copy(T* dst, const T* src, T s, long n) {
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
        dst[i] = s * src[i];
}

template <class T>
void launch_scale_copy(T* dst, const T* src, T s, long n, hipStream_t st) {
    long blocks = (n + PB - 1) / PB;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_scale_copy<T>, dim3(blocks), dim3(PB), 0, st, dst, src, s, n);
}

// ---------------------------------------------------------------------------
// kick / drift / tile key with wave-aggregated histogram atomics
// ---------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(PB) void k_kick_drift_key(Parts<T> p, SortBufs s, Geo g, T kick,
                                                       T drift, int mode, uint32_t* status) {
    const long n = g.npart;
    const int lane = threadIdx.x & 63;
    for (long base = blockIdx.x * (long)PB; base < n; base += (long)gridDim.x * PB) {
        long k = base + threadIdx.x;
        bool valid = k < n;
        uint32_t key = 0;
        if (valid) {
            T d[3], m[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                d[a] = p.disp[a * n + k];
                m[a] = p.mom[a * n + k];
            }
            if (mode & MODE_KICK) {
#pragma unroll
                for (int a = 0; a < 3; ++a) m[a] += kick * p.acc[a * n + k];
            }
            if (mode & MODE_DRIFT) {
#pragma unroll
                for (int a = 0; a < 3; ++a) d[a] += drift * m[a];
            }
            if (!finite3(d[0], d[1], d[2])) {
                atomicOr(status, 1u);
                d[0] = d[1] = d[2] = T(0);
            }
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                p.disp[a * n + k] = d[a];
                if (mode & MODE_KICK) p.mom[a * n + k] = m[a];
            }
            int i0, i1, i2;
            lattice_of(p.id[k], g.np, i0, i1, i2);
            int c0, c1, c2;
            T t;
            cell_of(g.B, i0, d[0], g.nm, c0, t);
            cell_of(g.B, i1, d[1], g.nm, c1, t);
            cell_of(g.B, i2, d[2], g.nm, c2, t);
            key = (uint32_t)(((c0 / TILE) * g.nt + c1 / TILE) * g.nt + c2 / TILE);
            s.key[k] = key;
        }
        // wave-aggregated rank assignment: one atomic per distinct key per wave
        bool pending = valid;
        uint32_t myrank = 0;
        while (__any(pending)) {
            unsigned long long m = __ballot(pending);
            int leader = __ffsll((long long)m) - 1;
            uint32_t lkey = __shfl(key, leader);
            bool mine = pending && key == lkey;
            unsigned long long same = __ballot(mine);
            uint32_t b0 = 0;
            if (lane == leader) b0 = atomicAdd(&s.count[lkey], (uint32_t)__popcll(same));
            b0 = __shfl(b0, leader);
            if (mine) {
                myrank = b0 + (uint32_t)__popcll(same & ((1ull << lane) - 1ull));
                pending = false;
            }
        }
        if (valid) s.rank[k] = myrank;
    }
}

template <class T>
void launch_kick_drift_key(Parts<T> p, SortBufs s, Geo g, T kick, T drift, int mode,
                           uint32_t* status, hipStream_t st) {
    long blocks = (g.npart + PB - 1) / PB;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_kick_drift_key<T>, dim3(blocks), dim3(PB), 0, st, p, s, g, kick, drift,
                       mode, status);
}

// ---------------------------------------------------------------------------
// exclusive scan of the tile histogram (one workgroup, chunk per thread)
// ---------------------------------------------------------------------------
constexpr int SCAN_T = 1024;
__global__ __launch_bounds__(SCAN_T) void k_scan(const uint32_t* count, uint32_t* start, int n) {
    __shared__ uint32_t part[SCAN_T];
    const int t = threadIdx.x;
    const int chunk = (n + SCAN_T - 1) / SCAN_T;
    const int lo = t * chunk;
    const int hi = min(n, lo + chunk);
    uint32_t sum = 0;
    for (int i = lo; i < hi; ++i) sum += count[i];
    part[t] = sum;
    __syncthreads();
    for (int off = 1; off < SCAN_T; off <<= 1) {
        uint32_t v = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t run = part[t] - sum;  // exclusive prefix of this chunk
    for (int i = lo; i < hi; ++i) {
        start[i] = run;
        run += count[i];
    }
    if (t == SCAN_T - 1) start[n] = part[t];
}

void launch_scan(const uint32_t* count, uint32_t* start, int n, hipStream_t st) {
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(SCAN_T), 0, st, count, start, n);
}

// ---------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(PB) void k_scatter(Parts<T> src, Parts<T> dst, SortBufs s, Geo g) {
    const long n = g.npart;
    for (long k = blockIdx.x * (long)PB + threadIdx.x; k < n; k += (long)gridDim.x * PB) {
        uint32_t d = s.start[s.key[k]] + s.rank[k];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            dst.disp[a * n + d] = src.disp[a * n + k];
            dst.mom[a * n + d] = src.mom[a * n + k];
        }
        dst.id[d] = src.id[k];
    }
}

template <class T>
void launch_scatter(Parts<T> src, Parts<T> dst, SortBufs s, Geo g, hipStream_t st) {
    long blocks = (g.npart + PB - 1) / PB;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_scatter<T>, dim3(blocks), dim3(PB), 0, st, src, dst, s, g);
}

// ---------------------------------------------------------------------------
// LDS-tiled CIC paint
// ---------------------------------------------------------------------------
__device__ __forceinline__ int halo_index(int x, int y, int z) {
    if (x == TILE) return y * TE + z;
    if (y == TILE) return TE * TE + x * TE + z;
    return TE * TE + TILE * TE + x * TILE + y;
}

__device__ __forceinline__ void halo_coords(int h, int& x, int& y, int& z) {
    if (h < TE * TE) { x = TILE; y = h / TE; z = h % TE; return; }
    h -= TE * TE;
    if (h < TILE * TE) { x = h / TE; y = TILE; z = h % TE; return; }
    h -= TILE * TE;
    x = h / TILE; y = h % TILE; z = TILE;
}

template <class T>
__global__ __launch_bounds__(PB) void k_paint_tile(Parts<T> p, SortBufs s, Geo g, T mass, T* rho,
                                                   T* halo) {
    __shared__ T tile[TE * TE * TE];
    const int tid = threadIdx.x;
    const int t = blockIdx.x;
    const int tx = t / (g.nt * g.nt), ty = (t / g.nt) % g.nt, tz = t % g.nt;
    const int ox = tx * TILE, oy = ty * TILE, oz = tz * TILE;
    for (int i = tid; i < TE * TE * TE; i += PB) tile[i] = T(0);
    __syncthreads();
    const long n = g.npart;
    const uint32_t lo = s.start[t], hi = s.start[t + 1];
    for (uint32_t k = lo + tid; k < hi; k += PB) {
        int i0, i1, i2;
        lattice_of(p.id[k], g.np, i0, i1, i2);
        int c0, c1, c2;
        T f0, f1, f2;
        cell_of(g.B, i0, p.disp[k], g.nm, c0, f0);
        cell_of(g.B, i1, p.disp[n + k], g.nm, c1, f1);
        cell_of(g.B, i2, p.disp[2 * n + k], g.nm, c2, f2);
        int l0 = min(max(c0 - ox, 0), TILE - 1);
        int l1 = min(max(c1 - oy, 0), TILE - 1);
        int l2 = min(max(c2 - oz, 0), TILE - 1);
        T w0[2] = {T(1) - f0, f0}, w1[2] = {T(1) - f1, f1}, w2[2] = {(T(1) - f2) * mass, f2 * mass};
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                T wab = w0[a] * w1[b];
                int base = ((l0 + a) * TE + (l1 + b)) * TE + l2;
                atomicAdd(&tile[base], wab * w2[0]);
                atomicAdd(&tile[base + 1], wab * w2[1]);
            }
    }
    __syncthreads();
    const long nm = g.nm;
    for (int i = tid; i < TILE * TILE * TILE; i += PB) {
        int x = i >> 8, y = (i >> 4) & 15, z = i & 15;
        rho[((ox + x) * nm + (oy + y)) * nm + (oz + z)] = tile[(x * TE + y) * TE + z];
    }
    for (int h = tid; h < HALO; h += PB) {
        int x, y, z;
        halo_coords(h, x, y, z);
        halo[(long)t * HALO + h] = tile[(x * TE + y) * TE + z];
    }
}

// Add the upper halo shells of the neighbouring tiles into the low faces of
// each tile (fixed order, no atomics).
template <class T>
__global__ __launch_bounds__(PB) void k_paint_halo(T* rho, const T* halo, Geo g) {
    const int t = blockIdx.x;
    const int nt = g.nt;
    const int tx = t / (nt * nt), ty = (t / nt) % nt, tz = t % nt;
    const long nm = g.nm;
    // 721 low-face cells: lx == 0 (256), ly == 0 && lx > 0 (240), lz == 0 && lx, ly > 0 (225)
    for (int f = threadIdx.x; f < 721; f += PB) {
        int lx, ly, lz;
        if (f < 256) { lx = 0; ly = f >> 4; lz = f & 15; }
        else if (f < 496) { int h = f - 256; lx = 1 + h / 16; ly = 0; lz = h % 16; }
        else { int h = f - 496; lx = 1 + h / 15; ly = 1 + h % 15; lz = 0; }
        T acc = T(0);
#pragma unroll
        for (int dx = 0; dx < 2; ++dx)
#pragma unroll
            for (int dy = 0; dy < 2; ++dy)
#pragma unroll
                for (int dz = 0; dz < 2; ++dz) {
                    if ((dx | dy | dz) == 0) continue;
                    if ((dx && lx) || (dy && ly) || (dz && lz)) continue;
                    int nx = tx - dx < 0 ? nt - 1 : tx - dx;
                    int ny = ty - dy < 0 ? nt - 1 : ty - dy;
                    int nz = tz - dz < 0 ? nt - 1 : tz - dz;
                    long nb = ((long)nx * nt + ny) * nt + nz;
                    acc += halo[nb * HALO + halo_index(lx + TILE * dx, ly + TILE * dy, lz + TILE * dz)];
                }
        long cell = ((long)(tx * TILE + lx) * nm + (ty * TILE + ly)) * nm + (tz * TILE + lz);
        rho[cell] += acc;
    }
}

template <class T>
void launch_paint(Parts<T> p, SortBufs s, Geo g, T mass, T* rho, T* halo, hipStream_t st) {
    int ntiles = g.nt * g.nt * g.nt;
    hipLaunchKernelGGL(k_paint_tile<T>, dim3(ntiles), dim3(PB), 0, st, p, s, g, mass, rho, halo);
    hipLaunchKernelGGL(k_paint_halo<T>, dim3(ntiles), dim3(PB), 0, st, rho, halo, g);
}

// ---------------------------------------------------------------------------
// LDS-staged CIC readout + kick
// ---------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(PB) void k_readout(Parts<T> p, SortBufs s, Geo g, const T* f0,
                                                const T* f1, const T* f2, T kick, int do_kick,
                                                uint32_t* status) {
    __shared__ T ft[3][TE * TE * TE];
    const int tid = threadIdx.x;
    const int t = blockIdx.x;
    const int tx = t / (g.nt * g.nt), ty = (t / g.nt) % g.nt, tz = t % g.nt;
    const int ox = tx * TILE, oy = ty * TILE, oz = tz * TILE;
    const uint32_t lo = s.start[t], hi = s.start[t + 1];
    if (lo == hi) return;  // uniform across the workgroup
    const int nm = g.nm;
    for (int i = tid; i < TE * TE * TE; i += PB) {
        int x = i / (TE * TE), y = (i / TE) % TE, z = i % TE;
        int gx = ox + x, gy = oy + y, gz = oz + z;
        if (gx >= nm) gx -= nm;
        if (gy >= nm) gy -= nm;
        if (gz >= nm) gz -= nm;
        long c = ((long)gx * nm + gy) * nm + gz;
        ft[0][i] = f0[c];
        ft[1][i] = f1[c];
        ft[2][i] = f2[c];
    }
    __syncthreads();
    const long n = g.npart;
    for (uint32_t k = lo + tid; k < hi; k += PB) {
        int i0, i1, i2;
        lattice_of(p.id[k], g.np, i0, i1, i2);
        T d0 = p.disp[k], d1 = p.disp[n + k], d2 = p.disp[2 * n + k];
        if (!finite3(d0, d1, d2)) atomicOr(status, 1u);
        int c0, c1, c2;
        T w0, w1, w2;
        cell_of(g.B, i0, d0, nm, c0, w0);
        cell_of(g.B, i1, d1, nm, c1, w1);
        cell_of(g.B, i2, d2, nm, c2, w2);
        int l0 = min(max(c0 - ox, 0), TILE - 1);
        int l1 = min(max(c1 - oy, 0), TILE - 1);
        int l2 = min(max(c2 - oz, 0), TILE - 1);
        T wa[2] = {T(1) - w0, w0}, wb[2] = {T(1) - w1, w1}, wc[2] = {T(1) - w2, w2};
        T a0 = 0, a1 = 0, a2 = 0;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                int base = ((l0 + a) * TE + (l1 + b)) * TE + l2;
                T wab = wa[a] * wb[b];
                T v0 = wab * wc[0], v1 = wab * wc[1];
                a0 += v0 * ft[0][base] + v1 * ft[0][base + 1];
                a1 += v0 * ft[1][base] + v1 * ft[1][base + 1];
                a2 += v0 * ft[2][base] + v1 * ft[2][base + 1];
            }
        p.acc[k] = a0;
        p.acc[n + k] = a1;
        p.acc[2 * n + k] = a2;
        if (do_kick) {
            p.mom[k] += kick * a0;
            p.mom[n + k] += kick * a1;
            p.mom[2 * n + k] += kick * a2;
        }
    }
}

template <class T>
void launch_readout(Parts<T> p, SortBufs s, Geo g, const T* f0, const T* f1, const T* f2,
                    T kick, int do_kick, uint32_t* status, hipStream_t st) {
    int ntiles = g.nt * g.nt * g.nt;
    hipLaunchKernelGGL(k_readout<T>, dim3(ntiles), dim3(PB), 0, st, p, s, g, f0, f1, f2, kick,
                       do_kick, status);
}

// ---------------------------------------------------------------------------
// initial conditions and state conversion
// ---------------------------------------------------------------------------
template <class T>
__global__ void k_init_ic(Parts<T> p, Geo g, const T* s0, const T* s1, const T* s2, T dfac,
                          T pfac) {
    const long n = g.npart;
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
        T v[3] = {s0[k], s1[k], s2[k]};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            p.disp[a * n + k] = dfac * v[a];
            p.mom[a * n + k] = pfac * v[a];
            p.acc[a * n + k] = T(0);
        }
        p.id[k] = (uint32_t)k;
    }
}

template <class T>
void launch_init_ic(Parts<T> p, Geo g, const T* s0, const T* s1, const T* s2, T dfac, T pfac,
                    hipStream_t st) {
    long blocks = (g.npart + PB - 1) / PB;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_init_ic<T>, dim3(blocks), dim3(PB), 0, st, p, g, s0, s1, s2, dfac, pfac);
}

template <class T>
__global__ void k_get_state(Parts<T> p, Geo g, T cell, T* x, T* mo, T* ac) {
    const long n = g.npart;
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
        uint32_t id = p.id[k];
        int i[3];
        lattice_of(id, g.np, i[0], i[1], i[2]);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (x) {
                int c;
                T f;
                cell_of(g.B, i[a], p.disp[a * n + k], g.nm, c, f);
                T v = (T(c) + f) * cell;
                if (v >= T(g.nm) * cell) v -= T(g.nm) * cell;
                x[a * n + id] = v;
            }
            if (mo) mo[a * n + id] = p.mom[a * n + k] * cell;
            if (ac) ac[a * n + id] = p.acc[a * n + k] * cell;
        }
    }
}

template <class T>
void launch_get_state(Parts<T> p, Geo g, T cell, T* x, T* mom_out, T* acc_out, hipStream_t st) {
    long blocks = (g.npart + PB - 1) / PB;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_get_state<T>, dim3(blocks), dim3(PB), 0, st, p, g, cell, x, mom_out, acc_out);
}

template <class T>
__global__ void k_set_state(Parts<T> p, Geo g, T cell, const T* x, const T* mi) {
    const long n = g.npart;
    const T nmf = T(g.nm);
    for (long k = blockIdx.x * (long)blockDim.x + threadIdx.x; k < n; k += (long)gridDim.x * blockDim.x) {
        int i[3];
        lattice_of((uint32_t)k, g.np, i[0], i[1], i[2]);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            T u = x[a * n + k] / cell;
            T d = u - (T(g.B * i[a]) + T(0.5));
            d -= nmf * floor(d / nmf + T(0.5));  // minimum image, [-nm/2, nm/2)
            p.disp[a * n + k] = d;
            p.mom[a * n + k] = mi[a * n + k] / cell;
            p.acc[a * n + k] = T(0);
        }
        p.id[k] = (uint32_t)k;
    }
}

template <class T>
void launch_set_state(Parts<T> p, Geo g, T cell, const T* x, const T* mom_in, hipStream_t st) {
    long blocks = (g.npart + PB - 1) / PB;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_set_state<T>, dim3(blocks), dim3(PB), 0, st, p, g, cell, x, mom_in);
}

#define ML_INST(T)                                                                                \
    template void launch_fill<T>(T*, T, long, hipStream_t);                                       \
    template void launch_scale_copy<T>(T*, const T*, T, long, hipStream_t);                       \
    template void launch_kick_drift_key<T>(Parts<T>, SortBufs, Geo, T, T, int, uint32_t*,        \
                                           hipStream_t);                                          \
    template void launch_scatter<T>(Parts<T>, Parts<T>, SortBufs, Geo, hipStream_t);              \
    template void launch_paint<T>(Parts<T>, SortBufs, Geo, T, T*, T*, hipStream_t);               \
    template void launch_readout<T>(Parts<T>, SortBufs, Geo, const T*, const T*, const T*, T, int, \
                                    uint32_t*, hipStream_t);                                      \
    template void launch_init_ic<T>(Parts<T>, Geo, const T*, const T*, const T*, T, T,            \
                                    hipStream_t);                                                 \
    template void launch_get_state<T>(Parts<T>, Geo, T, T*, T*, T*, hipStream_t);                 \
    template void launch_set_state<T>(Parts<T>, Geo, T, const T*, const T*, hipStream_t);
ML_INST(float)
ML_INST(double)

}  // namespace ml
