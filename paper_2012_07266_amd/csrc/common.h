// Shared device helpers of the MADLens HIP library: complex arithmetic,
// radix-2/3/4/8 DFT butterflies, periodic cell arithmetic for CIC.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ml {

template <class T> struct cx { T re, im; };

// Compiler-only fence: no memory access moves across it.  Used to keep
// loads that should be in flight together ahead of the LDS stores that
// consume them (and of branches that would delay their issue); it emits no
// instruction.
__device__ __forceinline__ void issue_fence() { asm volatile("" ::: "memory"); }

template <class T> __device__ __forceinline__ cx<T> mk(T r, T i) { return {r, i}; }
template <class T> __device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <class T> __device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <class T> __device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class T> __device__ __forceinline__ cx<T> scale(cx<T> a, T s) { return {a.re * s, a.im * s}; }
template <class T> __device__ __forceinline__ cx<T> conj(cx<T> a) { return {a.re, -a.im}; }
// multiply by -i*S (S = +1 forward, -1 inverse): (x + iy)(-iS) = S*y - i*S*x
template <int S, class T> __device__ __forceinline__ cx<T> mul_mi(cx<T> a) {
    return S > 0 ? cx<T>{a.im, -a.re} : cx<T>{-a.im, a.re};
}

// In-place R-point DFT with sign exp(-S 2 pi i nk/R), S = +1 forward.
template <int S, class T> __device__ __forceinline__ void dft2(cx<T>* u) {
    cx<T> a = u[0], b = u[1];
    u[0] = a + b;
    u[1] = a - b;
}

template <int S, class T> __device__ __forceinline__ void dft3(cx<T>* u) {
    const T c = T(-0.5);
    const T s = T(0.86602540378443864676372317075294);  // sqrt(3)/2
    cx<T> t = u[1] + u[2];
    cx<T> d = u[1] - u[2];
    cx<T> m = {u[0].re + c * t.re, u[0].im + c * t.im};
    // (-i S s) d
    cx<T> e = mul_mi<S>(d);
    e = scale(e, s);
    u[0] = u[0] + t;
    u[1] = m + e;
    u[2] = m - e;
}

template <int S, class T> __device__ __forceinline__ void dft4(cx<T>* u) {
    cx<T> t0 = u[0] + u[2];
    cx<T> t1 = u[0] - u[2];
    cx<T> t2 = u[1] + u[3];
    cx<T> t3 = mul_mi<S>(u[1] - u[3]);
    u[0] = t0 + t2;
    u[2] = t0 - t2;
    u[1] = t1 + t3;
    u[3] = t1 - t3;
}

template <int S, class T> __device__ __forceinline__ void dft8(cx<T>* u) {
    cx<T> e[4] = {u[0], u[2], u[4], u[6]};
    cx<T> o[4] = {u[1], u[3], u[5], u[7]};
    dft4<S>(e);
    dft4<S>(o);
    const T r = T(0.70710678118654752440084436210485);
    // w8^k = exp(-S i pi k / 4)
    cx<T> o1 = {r * (o[1].re + S * o[1].im), r * (o[1].im - S * o[1].re)};
    cx<T> o2 = mul_mi<S>(o[2]);
    cx<T> o3 = {r * (-o[3].re + S * o[3].im), r * (-o[3].im - S * o[3].re)};
    u[0] = e[0] + o[0];
    u[4] = e[0] - o[0];
    u[1] = e[1] + o1;
    u[5] = e[1] - o1;
    u[2] = e[2] + o2;
    u[6] = e[2] - o2;
    u[3] = e[3] + o3;
    u[7] = e[3] - o3;
}

template <int R, int S, class T> __device__ __forceinline__ void dft(cx<T>* u) {
    if constexpr (R == 2) dft2<S>(u);
    else if constexpr (R == 3) dft3<S>(u);
    else if constexpr (R == 4) dft4<S>(u);
    else dft8<S>(u);
}

// Floor of a real as int (values are far inside int range).
template <class T> __device__ __forceinline__ int ifloor(T v) {
    return (int)floor(v);
}

// Positive modulo for cell indices.
__device__ __forceinline__ int pmod(int a, int n) {
    int r = a % n;
    return r < 0 ? r + n : r;
}

}  // namespace ml
