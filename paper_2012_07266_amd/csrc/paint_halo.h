// Upper-shell layout of the CIC paint boxes and the sum that merges the
// shells into the low faces of the neighbouring boxes.  Shared by the paint
// kernels (which write the shells and can merge them in a pass of their
// own) and by the first r2c pass, which can merge them while it loads the
// rows of the density instead.
//
// A paint workgroup owns a group of G consecutive 16^3 tiles along axis 2:
// interior 16 x 16 x 16G cells, LDS box 17 x 17 x (16G+1).  Its upper shell
// is stored per group as the x-face [17][16G+1] (x = 16), the y-face
// [16][16G+1] (y = 16, x < 16) and the z-face [16][16] (z = 16G).  A cell with
// local coordinates (lx, ly, lz) receives, for every (dx, dy, dz) in {0,1}^3
// other than 0 with dx only where lx = 0 (and so on), the shell value at
// (lx + 16 dx, ly + 16 dy, lz + 16G dz) of the group (tx - dx, ty - dy,
// gz - dz), periodic.  The sum runs in a fixed order, so merging is
// deterministic wherever it happens.
#pragma once
#include "particles.h"

namespace ml {

template <int G> struct PaintBox {
    static constexpr int LZ = TILE * G;          // interior depth along axis 2
    static constexpr int EZ = LZ + 1;
    static constexpr int CELLS = TE * TE * EZ;
    static constexpr int HALO = 33 * EZ + TILE * TILE;  // x-face, y-face, z-face
};

template <int G>
__device__ __forceinline__ int halo_index_g(int x, int y, int z) {
    constexpr int EZ = PaintBox<G>::EZ;
    if (x == TILE) return y * EZ + z;
    if (y == TILE) return TE * EZ + x * EZ + z;
    return 33 * EZ + x * TILE + y;
}

template <int G>
__device__ __forceinline__ void halo_coords_g(int h, int& x, int& y, int& z) {
    constexpr int EZ = PaintBox<G>::EZ;
    if (h < TE * EZ) { x = TILE; y = h / EZ; z = h % EZ; return; }
    h -= TE * EZ;
    if (h < TILE * EZ) { x = h / EZ; y = TILE; z = h % EZ; return; }
    h -= TILE * EZ;
    x = h / TILE; y = h % TILE; z = PaintBox<G>::LZ;
}

// Sum of the neighbouring shells owed to mesh cell (X, Y, Z); 0 for cells
// off the low faces.  The seven candidate values are loaded first (each
// only where it is owed, else 0) and then summed in the fixed order
// (dx, dy, dz) = 001, 010, 011, 100, 101, 110, 111, so that a caller's loads
// are all in flight at once.
template <class T, int G>
__device__ __forceinline__ T halo_sum_g(const T* halo, int nt, int X, int Y, int Z) {
    using BX = PaintBox<G>;
    constexpr int LZ = BX::LZ;
    const int lx = X % TILE, ly = Y % TILE, lz = Z % LZ;
    if (lx && ly && lz) return T(0);
    const int tx = X / TILE, ty = Y / TILE, gz = Z / LZ, ng = nt / G;
    const int txm = tx == 0 ? nt - 1 : tx - 1;
    const int tym = ty == 0 ? nt - 1 : ty - 1;
    const int gzm = gz == 0 ? ng - 1 : gz - 1;
    T v[7];
#pragma unroll
    for (int d = 1; d < 8; ++d) {
        const int dx = d >> 2, dy = (d >> 1) & 1, dz = d & 1;
        const bool owed = (!dx || lx == 0) && (!dy || ly == 0) && (!dz || lz == 0);
        const long nb = ((long)(dx ? txm : tx) * nt + (dy ? tym : ty)) * ng + (dz ? gzm : gz);
        const int hi = halo_index_g<G>(lx + TILE * dx, ly + TILE * dy, lz + LZ * dz);
        // an index that is not owed may lie outside the buffer: never form it
        const long at = owed ? nb * BX::HALO + hi : 0;
        v[d - 1] = owed ? halo[at] : T(0);
    }
    T acc = T(0);
#pragma unroll
    for (int d = 0; d < 7; ++d) acc += v[d];
    return acc;
}

// Shells still to be merged into a painted mesh (halo == nullptr: none).
template <class T> struct HaloMerge {
    const T* halo = nullptr;
    int nt = 0;  // tiles per side
    int G = 1;   // tiles per paint group along axis 2
};

template <class T>
__device__ __forceinline__ T halo_sum(const HaloMerge<T>& hm, int X, int Y, int Z) {
    return hm.G == 2 ? halo_sum_g<T, 2>(hm.halo, hm.nt, X, Y, Z)
                     : halo_sum_g<T, 1>(hm.halo, hm.nt, X, Y, Z);
}

}  // namespace ml
