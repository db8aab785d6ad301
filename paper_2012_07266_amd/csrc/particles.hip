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
#include "paint_halo.h"
#include "batch.h"

namespace ml {

constexpr int PB = 256;  // threads per workgroup of the particle kernels

__device__ __forceinline__ void lattice_of(uint32_t id, int np, int& i0, int& i1, int& i2) {
    (void)np;
    i0 = (int)(id >> 20);
    i1 = (int)((id >> 10) & 1023u);
    i2 = (int)(id & 1023u);
}

// Base cell (wrapped) and fraction along one axis from the lattice index and
// the displacement.  The integer part of the lattice point stays exact.
template <class T>
__device__ __forceinline__ void cell_of(int B, int i, T disp, int nm, int& c, T& t) {
    T v = T(0.5) + disp;
    T fl = floor(v);
    t = v - fl;
    c = B * i + (int)fl;
    if ((unsigned)c >= (unsigned)nm) c = pmod(c, nm);
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

__global__ void k_fill_b(const FillArgs* __restrict__ tab) {
    const FillArgs a = tab[blockIdx.y];
    if (!a.on) return;
    for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < a.n; i += (long)gridDim.x * blockDim.x)
        a.p[i] = 0u;
}

void launch_fill_batch(const FillArgs* tab, long n_max, int slots, hipStream_t st) {
    long blocks = (n_max + PB - 1) / PB;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_fill_b, dim3(blocks, slots), dim3(PB), 0, st, tab);
}

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
// Tile of a particle displaced by d (cells) from its lattice point.
template <class T>
__device__ __forceinline__ uint32_t tile_key(uint32_t id, const T (&d)[3], const Geo& g) {
    int i0, i1, i2;
    lattice_of(id, g.np, i0, i1, i2);
    int c0, c1, c2;
    T t;
    cell_of(g.B, i0, d[0], g.nm, c0, t);
    cell_of(g.B, i1, d[1], g.nm, c1, t);
    cell_of(g.B, i2, d[2], g.nm, c2, t);
    return (uint32_t)(((c0 / TILE) * g.nt + c1 / TILE) * g.ncb + (c2 / TILE) * BPT +
                      (c0 % TILE) / KX);
}

// Histogram of the tile keys of the valid lanes: one atomic per distinct key
// per wave, whose result is not needed (no round trip).  Every lane of the
// wave must call it.
__device__ __forceinline__ void wave_count(bool valid, uint32_t key, uint32_t* count) {
    const int lane = threadIdx.x & 63;
    bool pending = valid;
    while (__any(pending)) {
        unsigned long long m = __ballot(pending);
        int leader = __ffsll((long long)m) - 1;
        uint32_t lkey = __shfl(key, leader);
        bool mine = pending && key == lkey;
        unsigned long long same = __ballot(mine);
        if (lane == leader) atomicAdd(&count[lkey], (uint32_t)__popcll(same));
        if (mine) pending = false;
    }
}

// Lanes of a wave grouped by key: the group's first lane (its leader) and,
// for each lane, the number of group members in lower lanes; the leader
// also holds the group size.  Arithmetic only (one ballot round per
// distinct key), no memory traffic.
struct WaveGroup {
    int leader;
    uint32_t before;  // group members in lower lanes
    uint32_t size;    // group size (leader lane only, else 0)
};

__device__ __forceinline__ WaveGroup wave_group(bool valid, uint32_t key) {
    const int lane = threadIdx.x & 63;
    WaveGroup w{0, 0u, 0u};
    bool pending = valid;
    while (__any(pending)) {
        unsigned long long m = __ballot(pending);
        int leader = __ffsll((long long)m) - 1;
        uint32_t lkey = __shfl(key, leader);
        bool mine = pending && key == lkey;
        unsigned long long same = __ballot(mine);
        if (mine) {
            w.leader = leader;
            w.before = (uint32_t)__popcll(same & ((1ull << lane) - 1ull));
            pending = false;
        }
        if (lane == leader) w.size = (uint32_t)__popcll(same);
    }
    return w;
}

// Rank of each valid lane among the particles of its tile, taken by counting
// the tile's histogram entry down: every group leader subtracts its group's
// size in the same atomic instruction, and the members number themselves
// below the returned value.  The ranks of a tile's particles are distinct and
// fill [0, count), and the histogram ends at zero, ready for the next step.
// Split in two so that several rank requests of one thread share a round
// trip: wave_take_issue for each, then wave_take_rank for each.  Every lane
// of the wave must call both.
__device__ __forceinline__ uint32_t wave_take_issue(const WaveGroup& w, uint32_t key,
                                                    uint32_t* count) {
    uint32_t top = 0;
    if (w.size) top = atomicSub(&count[key], w.size);
    return top;
}
__device__ __forceinline__ uint32_t wave_take_rank(const WaveGroup& w, uint32_t top) {
    return __shfl(top, w.leader) - 1u - w.before;
}

template <class T>
__global__ __launch_bounds__(PB) void k_kick_drift_key(Parts<T> p, SortBufs s, Geo g, T kick,
                                                       T drift, int mode, uint32_t* status) {
    const long n = g.npart;
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
            key = tile_key<T>(p.id[k], d, g);
            s.key[k] = key;
        }
        wave_count(valid, key, s.count);
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
constexpr int SCAN_T = 1024;  // counts per scan block (one per thread)

// Exclusive prefix sum of v over the 1024 threads of the block; *total gets
// the block's sum.  Wave-level shuffles, then the 16 wave sums in LDS.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* total) {
    __shared__ uint32_t ws[SCAN_T / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) ws[wid] = x;
    __syncthreads();
    if (wid == 0) {
        uint32_t w = lane < SCAN_T / 64 ? ws[lane] : 0u;
#pragma unroll
        for (int o = 1; o < SCAN_T / 64; o <<= 1) {
            uint32_t y = __shfl_up(w, o, 64);
            if (lane >= o) w += y;
        }
        if (lane < SCAN_T / 64) ws[lane] = w;
    }
    __syncthreads();
    *total = ws[SCAN_T / 64 - 1];
    return (wid ? ws[wid - 1] : 0u) + x - v;
}

// pass 1: every block scans its 1024 counts (coalesced) and records its sum
__device__ __forceinline__ void scan_blocks_body(const uint32_t* count, uint32_t* start,
                                                        uint32_t* block_sum, int n) {
    const int i = blockIdx.x * SCAN_T + threadIdx.x;
    uint32_t total;
    uint32_t e = block_exclusive_scan(i < n ? count[i] : 0u, &total);
    if (i < n) start[i] = e;
    if (threadIdx.x == 0) block_sum[blockIdx.x] = total;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_blocks(const uint32_t* count, uint32_t* start,
                                                        uint32_t* block_sum, int n) {
    scan_blocks_body(count, start, block_sum, n);
}
__global__ __launch_bounds__(SCAN_T) void k_scan_blocks_b(const ScanArgs* __restrict__ tab) {
    const ScanArgs a = tab[blockIdx.y];
    if (!a.on) return;
    scan_blocks_body(a.count, a.start, a.block_sum, a.n);
}

// pass 2: every block adds the sum of the blocks before it; the last one
// also writes start[n] (the particle count)
__device__ __forceinline__ void scan_add_body(uint32_t* start, const uint32_t* block_sum,
                                                     int n, int nblocks) {
    const int t = threadIdx.x;
    uint32_t total;
    // nblocks <= SCAN_T: one block sum per thread
    uint32_t off = block_exclusive_scan(t < nblocks ? block_sum[t] : 0u, &total);
    __shared__ uint32_t mine;
    if (t == (int)blockIdx.x) mine = off;
    __syncthreads();
    const int i = blockIdx.x * SCAN_T + t;
    if (i < n) start[i] += mine;
    if (blockIdx.x == nblocks - 1 && t == 0) start[n] = total;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_add(uint32_t* start, const uint32_t* block_sum,
                                                     int n, int nblocks) {
    scan_add_body(start, block_sum, n, nblocks);
}
__global__ __launch_bounds__(SCAN_T) void k_scan_add_b(const ScanArgs* __restrict__ tab,
                                                       int nblocks) {
    const ScanArgs a = tab[blockIdx.y];
    if (!a.on) return;
    scan_add_body(a.start, a.block_sum, a.n, nblocks);
}

void launch_scan_batch(const ScanArgs* tab, int n, int slots, hipStream_t st) {
    const int nb = (n + SCAN_T - 1) / SCAN_T;
    hipLaunchKernelGGL(k_scan_blocks_b, dim3(nb, slots), dim3(SCAN_T), 0, st, tab);
    hipLaunchKernelGGL(k_scan_add_b, dim3(nb, slots), dim3(SCAN_T), 0, st, tab, nb);
}

void launch_scan(const uint32_t* count, uint32_t* start, uint32_t* block_sum, int n,
                 hipStream_t st) {
    const int nb = (n + SCAN_T - 1) / SCAN_T;
    hipLaunchKernelGGL(k_scan_blocks, dim3(nb), dim3(SCAN_T), 0, st, count, start, block_sum, n);
    hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(SCAN_T), 0, st, start, block_sum, n, nb);
}

// ---------------------------------------------------------------------------
// Particles k = base + u * PB + thread (u < SU) of a scatter batch: keys,
// destinations and data are all loaded before the one atomic round trip of
// the batch's ranks.  Lanes past the end load the last particle (so that no
// load is conditional and the loads stay in flight together) and store
// nothing.
constexpr int SU = 4;

// With TAN the two tangent arrays of tc ([3][n] each) travel with the
// particles (the forward-mode pass keeps its tangents in tile order).
template <class T, bool TAN>
__device__ __forceinline__ void scatter_body(Parts<T> src, Parts<T> dst, SortBufs s, Geo g,
                                                TanCarry<T> tc) {
    const long n = g.npart;
    for (long base = blockIdx.x * (long)(PB * SU); base < n; base += (long)gridDim.x * PB * SU) {
        bool valid[SU];
        long kc[SU];
        uint32_t key[SU], first[SU], idv[SU], top[SU];
        T dv[SU][3], mv[SU][3], xv[TAN ? SU : 1][3], pv[TAN ? SU : 1][3];
        WaveGroup w[SU];
#pragma unroll
        for (int u = 0; u < SU; ++u) {
            const long k = base + u * PB + threadIdx.x;
            valid[u] = k < n;
            kc[u] = valid[u] ? k : n - 1;
            key[u] = s.key[kc[u]];
        }
#pragma unroll
        for (int u = 0; u < SU; ++u) {
            idv[u] = src.id[kc[u]];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                dv[u][a] = src.disp[a * n + kc[u]];
                mv[u][a] = src.mom[a * n + kc[u]];
                if constexpr (TAN) {
                    xv[u][a] = tc.x_src[a * n + kc[u]];
                    pv[u][a] = tc.p_src[a * n + kc[u]];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < SU; ++u) first[u] = s.start[key[u]];
#pragma unroll
        for (int u = 0; u < SU; ++u) w[u] = wave_group(valid[u], key[u]);
#pragma unroll
        for (int u = 0; u < SU; ++u) top[u] = wave_take_issue(w[u], key[u], s.count);
#pragma unroll
        for (int u = 0; u < SU; ++u) {
            const uint32_t r = wave_take_rank(w[u], top[u]);
            if (!valid[u]) continue;
            const uint32_t d = first[u] + r;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                dst.disp[a * n + d] = dv[u][a];
                dst.mom[a * n + d] = mv[u][a];
                if constexpr (TAN) {
                    tc.x_dst[a * n + d] = xv[u][a];
                    tc.p_dst[a * n + d] = pv[u][a];
                }
            }
            dst.id[d] = idv[u];
        }
    }
}

template <class T, bool TAN>
__global__ __launch_bounds__(PB) void k_scatter(Parts<T> src, Parts<T> dst, SortBufs s, Geo g,
                                                TanCarry<T> tc) {
    scatter_body<T, TAN>(src, dst, s, g, tc);
}
template <class T>
__global__ __launch_bounds__(PB) void k_scatter_b(const ScatterArgs<T>* __restrict__ tab) {
    const ScatterArgs<T> a = tab[blockIdx.y];
    if (!a.on) return;
    scatter_body<T, false>(a.src, a.dst, a.s, a.g, TanCarry<T>());
}

template <class T>
void launch_scatter(Parts<T> src, Parts<T> dst, SortBufs s, Geo g, hipStream_t st,
                    TanCarry<T> tc) {
    long blocks = (g.npart + PB * SU - 1) / (PB * SU);
    if (blocks > 16384) blocks = 16384;
    if (tc.x_src)
        hipLaunchKernelGGL((k_scatter<T, true>), dim3(blocks), dim3(PB), 0, st, src, dst, s, g, tc);
    else
        hipLaunchKernelGGL((k_scatter<T, false>), dim3(blocks), dim3(PB), 0, st, src, dst, s, g, tc);
}

// ---------------------------------------------------------------------------
// LDS-tiled CIC paint.  A workgroup owns a group of G consecutive tiles
// along axis 2 (16 x 16 x 16G cells; the sort key orders those tiles
// consecutively, so their particles form one contiguous range).  It paints
// into a 17 x 17 x (16G+1) LDS box, stores the 16 x 16 x 16G interior with
// plain stores and its upper shell (x = 16, y = 16 or z = 16G) to a halo
// buffer; a second kernel adds the shells into the low faces of the
// neighbouring groups in a fixed order.  The x and y faces are contiguous
// along axis 2, so both kernels move whole rows.
// ---------------------------------------------------------------------------
constexpr int PU = 4;    // particles per thread in flight
constexpr int PBP = 512; // threads per paint workgroup

// LDS accumulator of the paint box.  float: signed 64-bit fixed point (integer
// LDS atomics run at full rate on gfx950 while float ones do not, and the
// integer sum is exact and order-independent).  The scale is 2^32 for the
// density (weights <= 8) and 2^40 / max|value| (a power of two) when
// arbitrary values are painted.  double: float64 atomics.
template <class T> struct PaintAcc;
template <> struct PaintAcc<float> {
    using S = unsigned long long;
    static __device__ __forceinline__ S enc(float w, float scale) {
        return (S)__float2ll_rn(w * scale);
    }
    static __device__ __forceinline__ float dec(S v, double inv_scale) {
        return (float)((double)(long long)v * inv_scale);
    }
};
template <> struct PaintAcc<double> {
    using S = double;
    static __device__ __forceinline__ S enc(double w, double) { return w; }
    static __device__ __forceinline__ double dec(S v, double) { return v; }
};

// Fixed-point scale for painting values whose largest magnitude has the
// float bit pattern *vmax_bits (2^40 / max, rounded down to a power of two).
__device__ __forceinline__ float value_scale(const uint32_t* vmax_bits) {
    float m = __uint_as_float(*vmax_bits);
    if (!(m > 0.f) || !isfinite(m)) return 1.0f;
    int e = ilogbf(m) + 1;  // m < 2^e
    return ldexpf(1.0f, 40 - e);
}

// Particles k0, k0 + PBP, ... (PU of them, below hi) of a paint batch.  With
// TAN the three components of a tangent ([3][n], cells) go to tv.
template <class T, bool TAN>
__device__ __forceinline__ void paint_load_batch(const Parts<T>& p, long n, uint32_t k0,
                                                 uint32_t hi, const T* vals, T mass,
                                                 uint32_t (&idv)[PU], T (&dv)[PU][3],
                                                 T (&mv)[PU], T (&tv)[PU][3]) {
#pragma unroll
    for (int u = 0; u < PU; ++u) {
        uint32_t k = k0 + u * PBP;
        if (k < hi) {
            idv[u] = p.id[k];
            dv[u][0] = p.disp[k];
            dv[u][1] = p.disp[n + k];
            dv[u][2] = p.disp[2 * n + k];
            if constexpr (TAN) {
                tv[u][0] = vals[k];
                tv[u][1] = vals[n + k];
                tv[u][2] = vals[2 * n + k];
            } else {
                mv[u] = vals ? vals[k] : mass;
            }
        }
    }
}

// TAN: tangent paint, d/de of the density at x + e xdot for the tangent
// vals = xdot ([3][n] cells): corner c of a particle receives
// mass sum_a (dW_c/du_a) xdot_a (vmax_bits then bounds mass sum_a |xdot_a|).
template <class T, int G, bool TAN>
__device__ __forceinline__ void paint_group_body(Parts<T> p, SortBufs s, Geo g, T mass, T* rho,
                                                     T* halo, const T* vals,
                                                     const uint32_t* vmax_bits) {
    using BX = PaintBox<G>;
    using A = PaintAcc<T>;
    using S = typename A::S;
    __shared__ S box[BX::CELLS];
    const int tid = threadIdx.x;
    const int ng = g.nt / G;  // groups along axis 2
    const int grp = blockIdx.x;
    const int tx = grp / (g.nt * ng), ty = (grp / ng) % g.nt, gz = grp % ng;
    const int ox = tx * TILE, oy = ty * TILE, oz = gz * BX::LZ;
    const T scale = vals ? (T)value_scale(vmax_bits) : T(4294967296.0);
    const double inv_scale = 1.0 / (double)scale;
    const long n = g.npart;
    const int b0 = tile_block(g, tx, ty, gz * G);
    const uint32_t lo = s.start[b0], hi = s.start[b0 + G * BPT];
    uint32_t idv[PU];
    T dv[PU][3], mv[PU], tv[PU][3];
    // the first batch is in flight while the box is cleared
    paint_load_batch<T, TAN>(p, n, lo + tid, hi, vals, mass, idv, dv, mv, tv);
    for (int i = tid; i < BX::CELLS; i += PBP) box[i] = S(0);
    __syncthreads();
    for (uint32_t base = lo; base < hi; base += PBP * PU) {
        if (base != lo) paint_load_batch<T, TAN>(p, n, base + tid, hi, vals, mass, idv, dv, mv, tv);
#pragma unroll
        for (int u = 0; u < PU; ++u) {
            uint32_t k = base + u * PBP + tid;
            if (k >= hi) continue;
            int i0, i1, i2;
            lattice_of(idv[u], g.np, i0, i1, i2);
            int c0, c1, c2;
            T f0, f1, f2;
            cell_of(g.B, i0, dv[u][0], g.nm, c0, f0);
            cell_of(g.B, i1, dv[u][1], g.nm, c1, f1);
            cell_of(g.B, i2, dv[u][2], g.nm, c2, f2);
            int l0 = min(max(c0 - ox, 0), TILE - 1);
            int l1 = min(max(c1 - oy, 0), TILE - 1);
            int l2 = min(max(c2 - oz, 0), BX::LZ - 1);
            T w0[2] = {T(1) - f0, f0}, w1[2] = {T(1) - f1, f1};
            if constexpr (TAN) {
                // corner (a, b, c): w2[c] A_ab + dw2[c] B_ab with
                // A_ab = mass (dw0[a] w1[b] t0 + w0[a] dw1[b] t1),
                // B_ab = mass w0[a] w1[b] t2, dw = -1 (low) / +1 (high)
                const T t0 = mass * tv[u][0], t1 = mass * tv[u][1], t2 = mass * tv[u][2];
                const T w2[2] = {T(1) - f2, f2};
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b) {
                        const T d0 = a ? t0 : -t0, d1 = b ? t1 : -t1;
                        const T A_ = d0 * w1[b] + w0[a] * d1;
                        const T B_ = w0[a] * w1[b] * t2;
                        int cell = ((l0 + a) * TE + (l1 + b)) * BX::EZ + l2;
                        atomicAdd(&box[cell], A::enc(w2[0] * A_ - B_, scale));
                        atomicAdd(&box[cell + 1], A::enc(w2[1] * A_ + B_, scale));
                    }
            } else {
            T w2[2] = {(T(1) - f2) * mv[u], f2 * mv[u]};
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    T wab = w0[a] * w1[b];
                    int cell = ((l0 + a) * TE + (l1 + b)) * BX::EZ + l2;
                    atomicAdd(&box[cell], A::enc(wab * w2[0], scale));
                    atomicAdd(&box[cell + 1], A::enc(wab * w2[1], scale));
                }
            }
        }
    }
    __syncthreads();
    const long nm = g.nm;
    constexpr int NI = TILE * TILE * BX::LZ;
    for (int i = tid; i < NI; i += PBP) {
        int x = i / (TILE * BX::LZ), y = (i / BX::LZ) % TILE, z = i % BX::LZ;
        rho[((ox + x) * nm + (oy + y)) * nm + (oz + z)] =
            A::dec(box[(x * TE + y) * BX::EZ + z], inv_scale);
    }
    for (int h = tid; h < BX::HALO; h += PBP) {
        int x, y, z;
        halo_coords_g<G>(h, x, y, z);
        halo[(long)grp * BX::HALO + h] = A::dec(box[(x * TE + y) * BX::EZ + z], inv_scale);
    }
}

template <class T, int G, bool TAN>
__global__ __launch_bounds__(PBP) void k_paint_group(Parts<T> p, SortBufs s, Geo g, T mass, T* rho,
                                                     T* halo, const T* vals,
                                                     const uint32_t* vmax_bits) {
    paint_group_body<T, G, TAN>(p, s, g, mass, rho, halo, vals, vmax_bits);
}
template <class T, int G>
__global__ __launch_bounds__(PBP) void k_paint_group_b(const PaintArgs<T>* __restrict__ tab) {
    const PaintArgs<T> a = tab[blockIdx.y];
    if (!a.on) return;
    paint_group_body<T, G, false>(a.p, a.s, a.g, a.mass, a.rho, a.halo, nullptr, nullptr);
}

// Add the upper shells of the neighbouring groups into the low faces of each
// group (fixed order, no atomics).
template <class T, int G>
__global__ __launch_bounds__(PB) void k_paint_halo_group(T* rho, const T* halo, Geo g) {
    using BX = PaintBox<G>;
    constexpr int LZ = BX::LZ;
    const int grp = blockIdx.x;
    const int nt = g.nt, ng = nt / G;
    const int tx = grp / (nt * ng), ty = (grp / ng) % nt, gz = grp % ng;
    const long nm = g.nm;
    // low faces: lx == 0 (16 LZ), ly == 0 && lx > 0 (15 LZ), lz == 0 && lx, ly > 0 (225)
    constexpr int NF = 31 * LZ + 225;
    for (int f = threadIdx.x; f < NF; f += PB) {
        int lx, ly, lz;
        if (f < TILE * LZ) { lx = 0; ly = f / LZ; lz = f % LZ; }
        else if (f < 31 * LZ) { int h = f - TILE * LZ; lx = 1 + h / LZ; ly = 0; lz = h % LZ; }
        else { int h = f - 31 * LZ; lx = 1 + h / 15; ly = 1 + h % 15; lz = 0; }
        const int X = tx * TILE + lx, Y = ty * TILE + ly, Z = gz * LZ + lz;
        rho[((long)X * nm + Y) * nm + Z] += halo_sum_g<T, G>(halo, nt, X, Y, Z);
    }
}

int paint_group_size(int nt, int esize) {
    (void)esize;
    int G = 2;
    while (G > 1 && nt % G) G /= 2;
    return G;
}

long paint_halo_elems(int nt, int esize) {
    int G = paint_group_size(nt, esize);
    long groups = (long)nt * nt * (nt / G);
    long h = 33L * (TILE * G + 1) + TILE * TILE;
    return groups * h;
}

template <class T, bool TAN>
void launch_paint_group(Parts<T> p, SortBufs s, Geo g, T mass, T* rho, T* halo, const T* vals,
                        const uint32_t* vmax_bits, hipStream_t st, bool merge_halo) {
    int G = paint_group_size(g.nt, sizeof(T));
    int groups = g.nt * g.nt * (g.nt / G);
    if (G == 2) {
        hipLaunchKernelGGL((k_paint_group<T, 2, TAN>), dim3(groups), dim3(PBP), 0, st, p, s, g, mass,
                           rho, halo, vals, vmax_bits);
        if (merge_halo)
            hipLaunchKernelGGL((k_paint_halo_group<T, 2>), dim3(groups), dim3(PB), 0, st, rho, halo, g);
    } else {
        hipLaunchKernelGGL((k_paint_group<T, 1, TAN>), dim3(groups), dim3(PBP), 0, st, p, s, g, mass,
                           rho, halo, vals, vmax_bits);
        if (merge_halo)
            hipLaunchKernelGGL((k_paint_halo_group<T, 1>), dim3(groups), dim3(PB), 0, st, rho, halo, g);
    }
}

template <class T>
void launch_paint_values(Parts<T> p, SortBufs s, Geo g, T mass, T* rho, T* halo, const T* vals,
                         const uint32_t* vmax_bits, hipStream_t st, bool merge_halo) {
    launch_paint_group<T, false>(p, s, g, mass, rho, halo, vals, vmax_bits, st, merge_halo);
}

template <class T>
void launch_paint_tangent(Parts<T> p, SortBufs s, Geo g, T mass, T* rho, T* halo, const T* xdot,
                          const uint32_t* vmax_bits, hipStream_t st, bool merge_halo) {
    launch_paint_group<T, true>(p, s, g, mass, rho, halo, xdot, vmax_bits, st, merge_halo);
}

template <class T>
void launch_paint(Parts<T> p, SortBufs s, Geo g, T mass, T* rho, T* halo, hipStream_t st,
                  bool merge_halo) {
    launch_paint_values<T>(p, s, g, mass, rho, halo, nullptr, nullptr, st, merge_halo);
}

template <class T>
HaloMerge<T> paint_halo_merge(Geo g, const T* halo) {
    HaloMerge<T> hm;
    hm.halo = halo;
    hm.nt = g.nt;
    hm.G = paint_group_size(g.nt, sizeof(T));
    return hm;
}

// ---------------------------------------------------------------------------
// LDS-staged CIC readout + kick
// ---------------------------------------------------------------------------
// The readout works on one sort block (8 x 16 x 16 cells) per workgroup,
// with the block's 9 x 17 x 17 force values of each component in LDS
// (31 KB in float32).  The box's rows along axis 2, the contiguous one, keep
// their full 17 values, so the box costs hardly more memory requests per
// particle than a whole tile's 17^3 box, which fits only two workgroups per
// CU.  Four particles per thread in flight hold the kernel to four
// workgroups per CU (by registers): with five, their boxes in flight
// outgrow an XCD's L2 and the overlap rows are fetched again.
constexpr int PBR = 256;  // threads per readout workgroup
constexpr int PUR = 4;    // particles per readout thread in flight
constexpr int RX = KX + 1;  // LDS extents of the readout box: RX x TE x RZ
constexpr int RZ = TE;
constexpr int RC = RX * TE * RZ;  // LDS cells of the readout box

// Workgroups are handed to the 8 XCDs round-robin.  Renumber them so that
// each XCD walks a contiguous run of blocks: neighbouring blocks then share
// the 128-byte lines of their one-cell overlap in the same L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
    constexpr int NX = 8;
    if (nb % NX) return b;
    return (b % NX) * (nb / NX) + b / NX;
}

// CIC force at a particle (displacement d from lattice point id) from the
// LDS box of the three components at origin (ox, oy, oz).
template <class T>
__device__ __forceinline__ void tile_force(const Geo& g, uint32_t id, const T (&d)[3],
                                           const T (*ft)[RC], int ox, int oy, int oz,
                                           T& a0, T& a1, T& a2) {
    int i0, i1, i2;
    lattice_of(id, g.np, i0, i1, i2);
    int c0, c1, c2;
    T w0, w1, w2;
    cell_of(g.B, i0, d[0], g.nm, c0, w0);
    cell_of(g.B, i1, d[1], g.nm, c1, w1);
    cell_of(g.B, i2, d[2], g.nm, c2, w2);
    int l0 = min(max(c0 - ox, 0), KX - 1);
    int l1 = min(max(c1 - oy, 0), TILE - 1);
    int l2 = min(max(c2 - oz, 0), TILE - 1);
    T wa[2] = {T(1) - w0, w0}, wb[2] = {T(1) - w1, w1}, wc[2] = {T(1) - w2, w2};
    a0 = a1 = a2 = T(0);
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            int cb = ((l0 + a) * TE + (l1 + b)) * RZ + l2;
            T wab = wa[a] * wb[b];
            T v0 = wab * wc[0], v1 = wab * wc[1];
            a0 += v0 * ft[0][cb] + v1 * ft[0][cb + 1];
            a1 += v0 * ft[1][cb] + v1 * ft[1][cb + 1];
            a2 += v0 * ft[2][cb] + v1 * ft[2][cb + 1];
        }
}

// The gradient of the CIC readout of each component along ud, fg_j =
// ud . grad R(x, M_j), from the same LDS box: the operations, in the same
// order, of the derivative passes' gather (CIC derivative -1 to the low node
// and +1 to the high one along each axis).
template <class T>
__device__ __forceinline__ void tile_force_grad(const Geo& g, uint32_t id, const T (&d)[3],
                                                const T (*ft)[RC], int ox, int oy, int oz,
                                                const T (&ud)[3], T (&fg)[3]) {
    int i0, i1, i2;
    lattice_of(id, g.np, i0, i1, i2);
    int c0, c1, c2;
    T t0, t1, t2;
    cell_of(g.B, i0, d[0], g.nm, c0, t0);
    cell_of(g.B, i1, d[1], g.nm, c1, t1);
    cell_of(g.B, i2, d[2], g.nm, c2, t2);
    const int l0 = min(max(c0 - ox, 0), KX - 1);
    const int l1 = min(max(c1 - oy, 0), TILE - 1);
    const int l2 = min(max(c2 - oz, 0), TILE - 1);
    const T w[3][2] = {{T(1) - t0, t0}, {T(1) - t1, t1}, {T(1) - t2, t2}};
    const int base = (l0 * TE + l1) * RZ + l2;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        T gr[3] = {T(0), T(0), T(0)};
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const T m = ft[j][base + (a * TE + b) * RZ + c];
                    const T d0 = a ? T(1) : T(-1), d1 = b ? T(1) : T(-1), d2 = c ? T(1) : T(-1);
                    gr[0] += d0 * w[1][b] * w[2][c] * m;
                    gr[1] += w[0][a] * d1 * w[2][c] * m;
                    gr[2] += w[0][a] * w[1][b] * d2 * m;
                }
        fg[j] = ud[0] * gr[0] + ud[1] * gr[1] + ud[2] * gr[2];
    }
}

// Readout fused with the start of the next step: p += K2 f, then the next
// step's p += K1' f and disp += Dr' p, and the particle's new tile key and
// its histogram count (the work of k_kick_drift_key, with f still in
// registers).  The same
// operations in the same order as the separate kernels.
template <class T>
__device__ __forceinline__ void readout_kick_drift_key(
    Parts<T>& p, const SortBufs& s, const Geo& g, long n, uint32_t k, bool valid, uint32_t id,
    const T (&dv)[3], const T (&mv)[3], const T (*ft)[RC], int ox, int oy, int oz,
    T kick, const ReadoutNext<T>& nx, uint32_t* status) {
    uint32_t key = 0;
    if (valid) {
        if (!finite3(dv[0], dv[1], dv[2])) atomicOr(status, 1u);
        T f[3];
        tile_force<T>(g, id, dv, ft, ox, oy, oz, f[0], f[1], f[2]);
        T m[3], d[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            m[a] = mv[a] + kick * f[a];   // end of this step
            m[a] += nx.kick * f[a];       // first half-kick of the next
            d[a] = dv[a];
            d[a] += nx.drift * m[a];      // and its drift
        }
        if (!finite3(d[0], d[1], d[2])) {
            atomicOr(status, 1u);
            d[0] = d[1] = d[2] = T(0);
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            p.disp[a * n + k] = d[a];
            p.mom[a * n + k] = m[a];
        }
        key = tile_key<T>(id, d, g);
        s.key[k] = key;
    }
    wave_count(valid, key, s.count);
}

// Particles k0, k0 + PBR, ... (PUR of them) of a readout batch.  Slots at or
// past hi load particle hi - 1 instead (hi > lo, so it exists) and are not
// used: with no load conditional, the compiler keeps every load of the
// batch and of the force box in flight together.  Momenta are loaded even
// without a kick.
template <class T>
__device__ __forceinline__ void readout_load_batch(const Parts<T>& p, long n, uint32_t k0,
                                                   uint32_t hi, uint32_t (&idv)[PUR],
                                                   T (&dv)[PUR][3], T (&mv)[PUR][3]) {
#pragma unroll
    for (int u = 0; u < PUR; ++u) {
        uint32_t k = k0 + u * PBR;
        k = k < hi ? k : hi - 1u;
        idv[u] = p.id[k];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            dv[u][a] = p.disp[a * n + k];
            mv[u][a] = p.mom[a * n + k];
        }
    }
}

// TG: also the tangent's share (TanGather) for the plain readout.
template <class T, bool TG = false>
__device__ __forceinline__ void readout_body(Parts<T> p, SortBufs s, Geo g, const T* f0,
                                                const T* f1, const T* f2, T kick, int do_kick,
                                                uint32_t* status, ReadoutNext<T> nx,
                                                TanGather<T> tg = TanGather<T>()) {
    constexpr int TC = RC;
    __shared__ T ft[3][TC];
    const int tid = threadIdx.x;
    const int b0 = xcd_tile(blockIdx.x, gridDim.x);  // one sort block
    int ox, oy, oz;
    block_origin(g, b0, ox, oy, oz);
    const int nm = g.nm;
    const long n = g.npart;
    uint32_t idv[PUR];
    T dv[PUR][3], mv[PUR][3];
    // Issue order: the block's particle range and the force box (which does
    // not depend on it), then the first batch of particles, which waits
    // only for the range; then the force box goes to LDS.  The fences keep
    // this order (the compiler would otherwise test the range before issuing
    // the force loads, and move LDS stores, each waiting for its load, in
    // between the particle loads).
    const uint32_t lo = s.start[b0], hi = s.start[b0 + 1];
    {
        constexpr int IT = (TC + PBR - 1) / PBR;
        T v0[IT], v1[IT], v2[IT];
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            int i = tid + it * PBR;
            i = i < TC ? i : TC - 1;  // a repeat load, not stored
            {
                int x = i / (TE * RZ), y = (i / RZ) % TE, z = i % RZ;
                int gx = ox + x, gy = oy + y, gz = oz + z;
                if (gx >= nm) gx -= nm;
                if (gy >= nm) gy -= nm;
                if (gz >= nm) gz -= nm;
                long c = ((long)gx * nm + gy) * nm + gz;
                v0[it] = f0[c];
                v1[it] = f1[c];
                v2[it] = f2[c];
            }
        }
        issue_fence();
        if (lo == hi) return;  // uniform across the workgroup
        readout_load_batch<T>(p, n, lo + tid, hi, idv, dv, mv);
        issue_fence();
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            int i = tid + it * PBR;
            if (i < TC) {
                ft[0][i] = v0[it];
                ft[1][i] = v1[it];
                ft[2][i] = v2[it];
            }
        }
    }
    __syncthreads();
    float vmax = 0.f;  // TG: the tangent paint's bound over this block
    for (uint32_t base = lo; base < hi; base += PBR * PUR) {
        if (base != lo) readout_load_batch<T>(p, n, base + tid, hi, idv, dv, mv);
#pragma unroll
        for (int u = 0; u < PUR; ++u) {
            uint32_t k = base + u * PBR + tid;
            const bool valid = k < hi;
            if (nx.on) {  // wave-uniform: every lane takes part in the histogram
                readout_kick_drift_key<T>(p, s, g, n, k, valid, idv[u], dv[u], mv[u], ft, ox, oy,
                                          oz, kick, nx, status);
                continue;
            }
            if (!valid) continue;
            if (!finite3(dv[u][0], dv[u][1], dv[u][2])) atomicOr(status, 1u);
            T a0, a1, a2;
            tile_force<T>(g, idv[u], dv[u], ft, ox, oy, oz, a0, a1, a2);
            p.acc[k] = a0;
            p.acc[n + k] = a1;
            p.acc[2 * n + k] = a2;
            if (do_kick) {
                p.mom[k] = mv[u][0] + kick * a0;
                p.mom[n + k] = mv[u][1] + kick * a1;
                p.mom[2 * n + k] = mv[u][2] + kick * a2;
            }
            if constexpr (TG) {
                T ud[3], fg[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) ud[a] = tg.inv_h * tg.xdot[a * n + k];
                vmax = fmaxf(vmax, (float)(tg.mass * (fabs(ud[0]) + fabs(ud[1]) + fabs(ud[2]))));
                tile_force_grad<T>(g, idv[u], dv[u], ft, ox, oy, oz, ud, fg);
#pragma unroll
                for (int a = 0; a < 3; ++a) tg.fbc[a * n + k] = fg[a];
            }
        }
    }
    if constexpr (TG) {
        // one atomic per workgroup; a bound slightly above the maximum keeps
        // float rounding of the bound from under-sizing the fixed-point scale
        __shared__ float redv[PBR / 64];
        float v = vmax * 1.0001f;
        for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
        if ((tid & 63) == 0) redv[tid >> 6] = v;
        __syncthreads();
        if (tid == 0) {
            for (int i = 1; i < PBR / 64; ++i) v = fmaxf(v, redv[i]);
            if (v > 0.f) atomicMax(tg.vmax_bits, __float_as_uint(v));
        }
    }
}

template <class T>
__global__ __launch_bounds__(PBR) void k_readout(Parts<T> p, SortBufs s, Geo g, const T* f0,
                                                const T* f1, const T* f2, T kick, int do_kick,
                                                uint32_t* status, ReadoutNext<T> nx) {
    readout_body<T>(p, s, g, f0, f1, f2, kick, do_kick, status, nx);
}
template <class T>
__global__ __launch_bounds__(PBR) void k_readout_b(const ReadoutArgs<T>* __restrict__ tab) {
    const ReadoutArgs<T> a = tab[blockIdx.y];
    if (!a.on) return;
    readout_body<T>(a.p, a.s, a.g, a.f0, a.f1, a.f2, a.kick, a.do_kick, a.status, a.nx);
}

template <class T>
__global__ __launch_bounds__(PBR) void k_readout_tg(Parts<T> p, SortBufs s, Geo g, const T* f0,
                                                   const T* f1, const T* f2, T kick, int do_kick,
                                                   uint32_t* status, TanGather<T> tg) {
    readout_body<T, true>(p, s, g, f0, f1, f2, kick, do_kick, status, ReadoutNext<T>(), tg);
}

template <class T>
void launch_readout_tangent(Parts<T> p, SortBufs s, Geo g, const T* f0, const T* f1, const T* f2,
                            T kick, int do_kick, uint32_t* status, const TanGather<T>& tg,
                            hipStream_t st) {
    const int nblocks = g.nt * g.nt * g.ncb;
    hipLaunchKernelGGL(k_readout_tg<T>, dim3(nblocks), dim3(PBR), 0, st, p, s, g, f0, f1, f2, kick,
                       do_kick, status, tg);
}

template <class T>
void launch_readout(Parts<T> p, SortBufs s, Geo g, const T* f0, const T* f1, const T* f2,
                    T kick, int do_kick, uint32_t* status, hipStream_t st, ReadoutNext<T> nx) {
    const int nblocks = g.nt * g.nt * g.ncb;
    hipLaunchKernelGGL(k_readout<T>, dim3(nblocks), dim3(PBR), 0, st, p, s, g, f0, f1, f2, kick,
                       do_kick, status, nx);
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
        int i2 = (int)(k % g.np), i1 = (int)((k / g.np) % g.np), i0 = (int)(k / ((long)g.np * g.np));
        p.id[k] = pack_id(i0, i1, i2);
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
        uint32_t pid = p.id[k];
        long id = lattice_index(pid, g.np);
        int i[3];
        lattice_of(pid, g.np, i[0], i[1], i[2]);
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
        int i[3] = {(int)(k / ((long)g.np * g.np)), (int)((k / g.np) % g.np), (int)(k % g.np)};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            T u = x[a * n + k] / cell;
            T d = u - (T(g.B * i[a]) + T(0.5));
            d -= nmf * floor(d / nmf + T(0.5));  // minimum image, [-nm/2, nm/2)
            p.disp[a * n + k] = d;
            p.mom[a * n + k] = mi[a * n + k] / cell;
            p.acc[a * n + k] = T(0);
        }
        p.id[k] = pack_id(i[0], i[1], i[2]);
    }
}

template <class T>
void launch_set_state(Parts<T> p, Geo g, T cell, const T* x, const T* mom_in, hipStream_t st) {
    long blocks = (g.npart + PB - 1) / PB;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_set_state<T>, dim3(blocks), dim3(PB), 0, st, p, g, cell, x, mom_in);
}

// ---------------------------------------------------------------------------
// White noise from a counter-based generator: Philox4x64-10 (Salmon, Moraes,
// Dror, Shaw, SC 2011) keyed by (seed, 0); block c uses the counter
// (c + 1, 0, 0, 0) and yields 4 words, turned into uniforms (w >> 11) 2^-53
// and, pairwise, into 4 normals by Box-Muller: r = sqrt(-2 ln(1 - u0)),
// (r cos 2 pi u1, r sin 2 pi u1).  Element i of the lattice is normal i.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
    constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
        uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
        uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

template <class T>
__global__ void k_noise(T* out, long n, uint64_t key0, uint64_t key1) {
    const long nblk = (n + 3) / 4;
    for (long b = blockIdx.x * (long)blockDim.x + threadIdx.x; b < nblk;
         b += (long)gridDim.x * blockDim.x) {
        uint64_t c[4] = {(uint64_t)b + 1u, 0u, 0u, 0u};
        philox4x64_10(c, key0, key1);
        double z[4];
#pragma unroll
        for (int j = 0; j < 4; j += 2) {
            double u0 = (double)(c[j] >> 11) * 0x1.0p-53;
            double u1 = (double)(c[j + 1] >> 11) * 0x1.0p-53;
            double r = sqrt(-2.0 * log1p(-u0));
            double sn, cs;
            sincos(2.0 * 3.14159265358979323846 * u1, &sn, &cs);
            z[j] = r * cs;
            z[j + 1] = r * sn;
        }
        const long i0 = 4 * b;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (i0 + j < n) out[i0 + j] = (T)z[j];
    }
}

template <class T>
void launch_noise(T* out, long n, uint64_t seed, hipStream_t st) {
    long blocks = ((n + 3) / 4 + PB - 1) / PB;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_noise<T>, dim3(blocks), dim3(PB), 0, st, out, n, seed, (uint64_t)0);
}

template <class T>
void launch_scatter_batch(const ScatterArgs<T>* tab, const Geo& g, int slots, hipStream_t st) {
    long blocks = (g.npart + PB * SU - 1) / (PB * SU);
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL((k_scatter_b<T>), dim3(blocks, slots), dim3(PB), 0, st, tab);
}

template <class T>
void launch_paint_batch(const PaintArgs<T>* tab, const Geo& g, int slots, hipStream_t st) {
    const int G = paint_group_size(g.nt, sizeof(T));
    const int groups = g.nt * g.nt * (g.nt / G);
    if (G == 2)
        hipLaunchKernelGGL((k_paint_group_b<T, 2>), dim3(groups, slots), dim3(PBP), 0, st, tab);
    else
        hipLaunchKernelGGL((k_paint_group_b<T, 1>), dim3(groups, slots), dim3(PBP), 0, st, tab);
}

template <class T>
void launch_readout_batch(const ReadoutArgs<T>* tab, const Geo& g, int slots, hipStream_t st) {
    const int nblocks = g.nt * g.nt * g.ncb;
    hipLaunchKernelGGL(k_readout_b<T>, dim3(nblocks, slots), dim3(PBR), 0, st, tab);
}

#define ML_INST_BATCH(T)                                                                           \
    template void launch_scatter_batch<T>(const ScatterArgs<T>*, const Geo&, int, hipStream_t);   \
    template void launch_paint_batch<T>(const PaintArgs<T>*, const Geo&, int, hipStream_t);       \
    template void launch_readout_batch<T>(const ReadoutArgs<T>*, const Geo&, int, hipStream_t);
ML_INST_BATCH(float)
ML_INST_BATCH(double)

#define ML_INST(T)                                                                                \
    template void launch_fill<T>(T*, T, long, hipStream_t);                                       \
    template void launch_scale_copy<T>(T*, const T*, T, long, hipStream_t);                       \
    template void launch_kick_drift_key<T>(Parts<T>, SortBufs, Geo, T, T, int, uint32_t*,        \
                                           hipStream_t);                                          \
    template void launch_scatter<T>(Parts<T>, Parts<T>, SortBufs, Geo, hipStream_t, TanCarry<T>); \
    template void launch_paint<T>(Parts<T>, SortBufs, Geo, T, T*, T*, hipStream_t, bool);         \
    template void launch_paint_values<T>(Parts<T>, SortBufs, Geo, T, T*, T*, const T*,            \
                                         const uint32_t*, hipStream_t, bool);                     \
    template void launch_paint_tangent<T>(Parts<T>, SortBufs, Geo, T, T*, T*, const T*,           \
                                          const uint32_t*, hipStream_t, bool);                    \
    template HaloMerge<T> paint_halo_merge<T>(Geo, const T*);                                     \
    template void launch_readout<T>(Parts<T>, SortBufs, Geo, const T*, const T*, const T*, T, int, \
                                    uint32_t*, hipStream_t, ReadoutNext<T>);                      \
    template void launch_readout_tangent<T>(Parts<T>, SortBufs, Geo, const T*, const T*,          \
                                            const T*, T, int, uint32_t*, const TanGather<T>&,     \
                                            hipStream_t);                                         \
    template void launch_init_ic<T>(Parts<T>, Geo, const T*, const T*, const T*, T, T,            \
                                    hipStream_t);                                                 \
    template void launch_get_state<T>(Parts<T>, Geo, T, T*, T*, T*, hipStream_t);                 \
    template void launch_set_state<T>(Parts<T>, Geo, T, const T*, const T*, hipStream_t);    \
    template void launch_noise<T>(T*, long, uint64_t, hipStream_t);
ML_INST(float)
ML_INST(double)

}  // namespace ml
