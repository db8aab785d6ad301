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

// The seven shell values that may be owed to mesh cell (X, Y, Z), in the
// order (dx, dy, dz) = 001, 010, 011, 100, 101, 110, 111; 0 where nothing is
// owed.  Loads only; a caller can fetch several cells before summing.
template <class T, int G>
__device__ __forceinline__ void halo_fetch_g(const T* halo, int nt, int X, int Y, int Z, T (&v)[7]) {
    using BX = PaintBox<G>;
    constexpr int LZ = BX::LZ;
    const int lx = X % TILE, ly = Y % TILE, lz = Z % LZ;
    const int tx = X / TILE, ty = Y / TILE, gz = Z / LZ, ng = nt / G;
    const int txm = tx == 0 ? nt - 1 : tx - 1;
    const int tym = ty == 0 ? nt - 1 : ty - 1;
    const int gzm = gz == 0 ? ng - 1 : gz - 1;
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
}

template <class T>
__device__ __forceinline__ T halo_add(const T (&v)[7]) {
    T acc = T(0);
#pragma unroll
    for (int d = 0; d < 7; ++d) acc += v[d];
    return acc;
}

// Sum of the neighbouring shells owed to mesh cell (X, Y, Z) (0 for cells
// off the low faces), summed in the fixed order above.
template <class T, int G>
__device__ __forceinline__ T halo_sum_g(const T* halo, int nt, int X, int Y, int Z) {
    constexpr int LZ = PaintBox<G>::LZ;
    if ((X % TILE) && (Y % TILE) && (Z % LZ)) return T(0);
    T v[7];
    halo_fetch_g<T, G>(halo, nt, X, Y, Z, v);
    return halo_add<T>(v);
}

// Shells still to be merged into a painted mesh (halo == nullptr: none).
template <class T> struct HaloMerge {
    const T* halo = nullptr;
    int nt = 0;  // tiles per side
    int G = 1;   // tiles per paint group along axis 2
};

// Add the shells owed to the rows X, Y0 .. Y0 + W - 1 (all 2H cells along
// axis 2 each) held in LDS as buf[(Z / 2) * LD + w] (.re: even Z, .im: odd
// Z).  Only the owed cells are visited: every cell when X is on a tile's low
// face, else the whole row on a tile's low y-face and the low z-face cells
// of the others.  Each thread fetches BATCH cells before summing any, so its
// loads are in flight together.  Ends with a barrier.
template <class T, int G, int H, int W, int NTT>
__device__ __forceinline__ void merge_rows_g(const HaloMerge<T>& hm, cx<T>* buf, int X, int Y0,
                                             int tid) {
    constexpr int LD = W + 1, NZ = 2 * H, LZ = PaintBox<G>::LZ, BATCH = 4;
    const bool all = (X % TILE) == 0;
    int wy = -1;  // the row on a tile's low y-face, if any
    for (int w = 0; w < W; ++w)
        if ((Y0 + w) % TILE == 0) wy = w;
    const int nz_face = NZ / LZ;
    const int owed = all ? W * NZ : (wy >= 0 ? NZ + (W - 1) * nz_face : W * nz_face);
    for (int c0 = tid; c0 < owed; c0 += NTT * BATCH) {
        T v[BATCH][7];
        int ws[BATCH], zs[BATCH];
#pragma unroll
        for (int b = 0; b < BATCH; ++b) {
            const int c = c0 + b * NTT;
            int w = 0, z = 0;
            if (all) {
                w = c / NZ;
                z = c % NZ;
            } else if (wy >= 0 && c < NZ) {
                w = wy;
                z = c;
            } else {
                const int e = wy >= 0 ? c - NZ : c;  // among the other rows
                const int r = e / nz_face;
                w = (wy >= 0 && r >= wy) ? r + 1 : r;
                z = (e % nz_face) * LZ;
            }
            ws[b] = w;
            zs[b] = z;
            if (c < owed) halo_fetch_g<T, G>(hm.halo, hm.nt, X, Y0 + w, z, v[b]);
        }
#pragma unroll
        for (int b = 0; b < BATCH; ++b) {
            if (c0 + b * NTT >= owed) continue;
            const T add = halo_add<T>(v[b]);
            cx<T>& e = buf[(zs[b] >> 1) * LD + ws[b]];
            if (zs[b] & 1) e.im += add;
            else e.re += add;
        }
    }
    __syncthreads();
}

template <class T, int H, int W, int NTT>
__device__ __forceinline__ void merge_rows(const HaloMerge<T>& hm, cx<T>* buf, int X, int Y0,
                                           int tid) {
    if (hm.G == 2) merge_rows_g<T, 2, H, W, NTT>(hm, buf, X, Y0, tid);
    else merge_rows_g<T, 1, H, W, NTT>(hm, buf, X, Y0, tid);
}

}  // namespace ml
