// Host entry points of the particle kernels (see particles.hip, lens.hip).
#pragma once
#include "common.h"

namespace ml {

constexpr int TILE = 16;                         // mesh cells per tile side
constexpr int TE = TILE + 1;                     // LDS tile side incl. +1 halo
constexpr int HALO = TE * TE + TILE * TE + TILE * TILE;  // 817 upper-shell cells

// Particle-lattice and mesh geometry.  Positions are stored as displacements
// from the lattice point in mesh-cell units; the lattice point of particle
// (i0, i1, i2) is u = B*i + 1/2 cells.
// Particles are sorted by blocks of KX x TILE x TILE cells (the key): a
// 16^3 tile is its two halves along axis 0, numbered consecutively, and the
// tiles of a column along axis 2 follow each other, so any run of tiles
// along axis 2 is one index range.
constexpr int BPT = 2;           // sort blocks per tile
constexpr int KX = TILE / BPT;   // extent of a sort block along axis 0

struct Geo {
    int np;      // particles per side
    int nm;      // mesh cells per side
    int B;       // nm / np
    int nt;      // tiles per side = nm / TILE
    long npart;  // np^3
    int ncb;     // sort blocks per tile column along axis 2 = nt * BPT
};

// Cell origin of sort block b (KX x TILE x TILE cells).
__host__ __device__ __forceinline__ void block_origin(const Geo& g, int b, int& ox, int& oy,
                                                      int& oz) {
    const int tx = b / (g.nt * g.ncb), ty = (b / g.ncb) % g.nt, kz = b % g.ncb;
    ox = tx * TILE + (kz % BPT) * KX;
    oy = ty * TILE;
    oz = (kz / BPT) * TILE;
}

// Index of the first sort block of tile (tx, ty, tz); the tile's particles
// are start[b] .. start[b + BPT].
__host__ __device__ __forceinline__ int tile_block(const Geo& g, int tx, int ty, int tz) {
    return (tx * g.nt + ty) * g.ncb + tz * BPT;
}

// Particle state in tile-sorted order (SoA, [3][npart] each).
template <class T> struct Parts {
    T* disp;        // displacement from the lattice point, cells
    T* mom;         // momentum, cells (p / H)
    T* acc;         // force at the particle, cells (f / H)
    uint32_t* id;   // packed lattice coordinates, see pack_id
};

struct SortBufs {
    uint32_t* key;    // tile of each particle
    uint32_t* count;  // [ntiles] histogram (zero between sorts)
    uint32_t* start;  // [ntiles+1] exclusive prefix
};

enum { MODE_KICK = 1, MODE_DRIFT = 2 };

// Particle ids pack the lattice coordinates (i0, i1, i2), each < 1024, as
// i0 << 20 | i1 << 10 | i2.
__device__ __forceinline__ uint32_t pack_id(int i0, int i1, int i2) {
    return ((uint32_t)i0 << 20) | ((uint32_t)i1 << 10) | (uint32_t)i2;
}
__device__ __forceinline__ void lattice_of_l(uint32_t id, int np, int* i) {
    (void)np;
    i[0] = (int)(id >> 20);
    i[1] = (int)((id >> 10) & 1023u);
    i[2] = (int)(id & 1023u);
}
// position in lattice order, (i0 * np + i1) * np + i2
__device__ __forceinline__ long lattice_index(uint32_t id, int np) {
    return ((long)(id >> 20) * np + ((id >> 10) & 1023u)) * np + (id & 1023u);
}

template <class T>
void launch_fill(T* p, T v, long n, hipStream_t st);
// dst[i] = s * src[i]
template <class T>
void launch_scale_copy(T* dst, const T* src, T s, long n, hipStream_t st);
void launch_fill_u32(uint32_t* p, uint32_t v, long n, hipStream_t st);

// mom += kick*acc (MODE_KICK), disp += drift*mom (MODE_DRIFT); then tile
// key and histogram of every particle.  `count` must be zero.
template <class T>
void launch_kick_drift_key(Parts<T> p, SortBufs s, Geo g, T kick, T drift, int mode,
                           uint32_t* status, hipStream_t st);
// Exclusive prefix sum of count[0..n) into start[0..n], start[n] = total;
// block_sum: scratch of (n + 1023) / 1024 entries (n <= 1024 * 1024).
void launch_scan(const uint32_t* count, uint32_t* start, uint32_t* block_sum, int n,
                 hipStream_t st);
// Tangent arrays ([3][npart], tile order) that a scatter carries with the
// particles: x_src -> x_dst and p_src -> p_dst.  x_src == NULL carries none.
template <class T> struct TanCarry {
    const T* x_src = nullptr;
    T* x_dst = nullptr;
    const T* p_src = nullptr;
    T* p_dst = nullptr;
};
// Permute disp, mom and id (and the tangents of tc) into tile order (dst),
// after launch_scan: each particle takes a rank in its tile by counting the
// histogram down, which leaves `count` at zero.
template <class T>
void launch_scatter(Parts<T> src, Parts<T> dst, SortBufs s, Geo g, hipStream_t st,
                    TanCarry<T> tc = TanCarry<T>());
// CIC paint of tile-sorted particles by groups of tiles along axis 2:
// interior cells go to rho, each group's upper halo shell to `halo` (size
// paint_halo_elems); then the shells are added into the neighbours' faces,
// unless merge_halo is false: the caller then merges them while reading rho
// (fft_r2c_rows with paint_halo_merge).
int paint_group_size(int nt, int esize);
long paint_halo_elems(int nt, int esize);
template <class T>
void launch_paint(Parts<T> p, SortBufs s, Geo g, T mass, T* rho, T* halo, hipStream_t st,
                  bool merge_halo = true);
// Paint per-particle values vals[k] (tile-sorted order) instead of the
// mass; *vmax_bits holds the float bits of max|vals| (sets the fixed-point
// scale of the float instantiation).
template <class T>
void launch_paint_values(Parts<T> p, SortBufs s, Geo g, T mass, T* rho, T* halo, const T* vals,
                         const uint32_t* vmax_bits, hipStream_t st, bool merge_halo = true);
// Tangent paint: d/de of the CIC density at x + e xdot, xdot [3][n] in
// tile-sorted order and cells; corner c of a particle receives
// mass sum_a (dW_c/du_a) xdot_a.  *vmax_bits holds the float bits of a bound
// of mass sum_a |xdot_a| over the particles (the fixed-point scale).
template <class T>
void launch_paint_tangent(Parts<T> p, SortBufs s, Geo g, T mass, T* rho, T* halo, const T* xdot,
                          const uint32_t* vmax_bits, hipStream_t st, bool merge_halo = true);
template <class T> struct HaloMerge;
// The shells of the last paint into `halo`, for a merge during the r2c pass.
template <class T>
HaloMerge<T> paint_halo_merge(Geo g, const T* halo);
// With `on`, the readout also starts the next step: after mom += kick*f it
// applies mom += kick'*f and disp += drift'*mom and writes the particles'
// tile keys and histogram (count must be zero), as launch_kick_drift_key would;
// acc is then not written.
template <class T> struct ReadoutNext {
    int on = 0;
    T kick = T(0);   // K1 of the next step
    T drift = T(0);  // Dr of the next step
};
// CIC readout of the three force meshes; acc = f; mom += kick*acc if do_kick.
template <class T>
void launch_readout(Parts<T> p, SortBufs s, Geo g, const T* f0, const T* f1, const T* f2,
                    T kick, int do_kick, uint32_t* status, hipStream_t st,
                    ReadoutNext<T> nx = ReadoutNext<T>());
// The tangent's share of a readout: the gradient of the CIC readout of each
// force mesh along u_dot = inv_h x_dot (x_dot [3][n] in Mpc/h, tile order),
// fbc_j = u_dot . grad R(x, M_j) (cells), and a bound of
// mass sum_a |u_dot_a| (the tangent paint's fixed-point scale) raised into
// *vmax_bits (float bits; the caller zeroes it).
template <class T> struct TanGather {
    const T* xdot = nullptr;
    T* fbc = nullptr;
    uint32_t* vmax_bits = nullptr;
    T inv_h = T(0);
    T mass = T(0);
};
// launch_readout (without the next step's kick and drift) that also
// computes the tangent's share of the same force meshes.
template <class T>
void launch_readout_tangent(Parts<T> p, SortBufs s, Geo g, const T* f0, const T* f1, const T* f2,
                            T kick, int do_kick, uint32_t* status, const TanGather<T>& tg,
                            hipStream_t st);
// Zel'dovich: disp = dfac*s, mom = pfac*s from the three displacement meshes
// on the particle lattice (cells), id = lattice index.
template <class T>
void launch_init_ic(Parts<T> p, Geo g, const T* s0, const T* s1, const T* s2, T dfac, T pfac,
                    hipStream_t st);
// State out in lattice order: x in [0, box) and p (Mpc/h), acc (Mpc/h).
template <class T>
void launch_get_state(Parts<T> p, Geo g, T cell, T* x, T* mom_out, T* acc_out, hipStream_t st);
// State in (lattice order, Mpc/h) -> displacement (minimum image), momentum.
template <class T>
void launch_set_state(Parts<T> p, Geo g, T cell, const T* x, const T* mom_in, hipStream_t st);
// N(0,1) noise [n] from Philox4x64-10 keyed by (seed, 0) and Box-Muller
template <class T>
void launch_noise(T* out, long n, uint64_t seed, hipStream_t st);

// Born projection of one shell (lens.hip).
constexpr int MAX_SRC = 16;
template <class T> struct LensArgs {
    int npix, nsrc;
    T cell;             // mesh cell size, Mpc/h
    T chi_near, chi_far;
    double cnear_d, cfar_d;  // the shell's depth bounds in cells, float64 (membership)
    T inv_dtheta;       // 1 / pixel size (radians)
    T wbase;            // 3/2 Om (H0/c)^2 V_p / Omega_pix
    T chi_src[MAX_SRC];
    const T* atab;      // [ntab][2]: a(chi_k), da/dchi(chi_k) at chi_k = k * dchi
    int ntab;
    T dchi;
    int rs;             // region side (pixels) of the gather projection
    // The region's LDS accumulators.  Map s takes its weight
    // w (cs - chi) / cs from every image in front of its source: slot[s] >= 0
    // is its own accumulator; slot[s] == -1 (dec != 0: two or more sources
    // beyond the shell's far bound, so that every image is in front of them)
    // is built at the end as A - ratio[s] B from the shared accumulators
    // A = sum w, B = sum w chi / chi_ref (slots 0 and 1), ratio = chi_ref / cs;
    // slot[s] == -2 takes nothing (its source is in front of the shell).
    // ndirect sources have their own slot, 2 dec + d, source direct_src[d].
    int dec, nacc, ndirect;
    int slot[MAX_SRC];
    int direct_src[MAX_SRC];
    double ratio[MAX_SRC];
    T inv_chi_ref;
    // sub-evolution (sub != 0): an image keeps the shell of its end-of-step
    // depth and moves by (D(a(chi)) - d_end) * sub_scale * p_h, p_h = mom -
    // sub_k2 * acc being the step's drift momentum (cells)
    int sub;
    const T* dtab;      // [ntab][2]: D(a(chi_k)), dD/dchi, on the atab grid
    T d_end;            // D at the end of the step
    T sub_scale;        // 1 / g_p(a_h)
    T sub_k2;           // 0: mom is the drift momentum; else mom - sub_k2 acc
    T sub_dr;           // the step's drift factor: bound of the move per |p_h|
    const uint32_t* pmax_bits;  // max |p_h| over particles and axes (float bits)
    int dwin;           // entries of dtab the kernel may copy to LDS (set by the launcher)
    // PGD: every image is shifted by shift_scale * shift[a * npart + k]
    // (cells) from its wrapped position before anything else (NULL: none);
    // *shift_bits holds max |shift| as float bits, for the frustum margin
    const T* shift;
    T shift_scale;
    const uint32_t* shift_bits;
    // replica rotation (rot != 0): replica (nx, ny, nz) is the box under one
    // of the 48 cube symmetries, hashed from its offsets and rot_seed
    int rot;
    unsigned long long rot_seed;
};
template <class T> struct MapAdd { T v[MAX_SRC]; };

// Shell membership.  An image's depth is its in-box coordinate along axis 2,
// an integer cell c plus a fraction f in [0, 1), plus nz Nm for replica nz.
// A depth bound (float64 cells) is moved into the replica's box and split the
// same way, so that comparing the pairs decides "depth > bound" exactly for
// the stored position, whatever the size of nz Nm: a float32 depth of ~2000
// cells would carry 1e-4 cells of rounding, far above the positions' own
// accuracy, and an image that changes sides moves its whole weight from one
// shell to the next.
template <class T> struct ZBound {
    int c;
    T f;
};
template <class T>
__device__ __forceinline__ ZBound<T> zbound(double b, int nz, int nm) {
    const double r = b - (double)nz * (double)nm;
    const double fl = floor(r);
    return {(int)fl, (T)(r - fl)};
}
template <class T>
__device__ __forceinline__ bool depth_in_shell(int c, T f, ZBound<T> lo, ZBound<T> hi) {
    const bool above = c > lo.c || (c == lo.c && f > lo.f);
    const bool at_most = c < hi.c || (c == hi.c && f <= hi.f);
    return above && at_most;
}
// The (cell, fraction) split of a float in-box coordinate.
template <class T>
__device__ __forceinline__ void split_cell(T u, int& c, T& f) {
    const T fl = floor(u);
    c = (int)fl;
    f = u - fl;
}
// Region-driven projection (each pixel written by one workgroup) that also
// adds mean.v[s] to every pixel of map s.  Particles must be tile-sorted.
template <class T>
void launch_lens_gather(Parts<T> p, SortBufs sb, Geo g, const LensArgs<T>& la,
                        const MapAdd<T>& mean, T* kappa, hipStream_t st);
// *out (zeroed by the caller) = bits of max |mom - k2 acc| over all
// particles and axes, as a float rounded up
template <class T>
void launch_drift_momentum_max(Parts<T> p, long n, T k2, uint32_t* out, hipStream_t st);


}  // namespace ml
