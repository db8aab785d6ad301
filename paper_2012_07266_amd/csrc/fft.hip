// LDS-staged Stockham FFT passes for 3D real meshes on gfx950, and the
// fused Fourier Poisson/gradient pass of the particle-mesh force.
//
// A real Nm^3 mesh (C order, last axis contiguous) is transformed in three
// 1D passes.  Its half spectrum is stored as
//   main [Nm][Nm][Nm/2]  complex, k2 = 0 .. Nm/2-1, in the same memory as
//                        the real mesh (rows of Nm reals = Nm/2 complex),
//   nyq  [Nm][Nm]        complex, the k2 = Nm/2 plane, in a side buffer,
// so every row of the main block stays 2 KB aligned for Nm = 512.
//
//   pass 1  r2c along axis 2: one row of Nm reals is packed into Nm/2
//           complex values, transformed, and split into Nm/2+1 outputs.
//   pass 2  c2c along axis 1 on main and nyq.
//   pass 3  fused along axis 0: forward transform, multiply by
//           i n_j G(|n|^2) for the three gradient components, inverse
//           transform each, write three spectra (one over the input).
//   pass 4  inverse c2c along axis 1 (three spectra).
//   pass 5  c2r along axis 2 (three spectra -> three real meshes in place).
//
// Each workgroup holds W pencils of one pass in LDS as [N][W+1] complex
// (the +1 pad keeps both row loads and column butterflies free of bank
// conflicts) and runs a mixed-radix (8, 4, 2, 3) Stockham transform in
// place: every stage reads its butterfly inputs into registers, barriers,
// and writes its outputs in natural-order Stockham positions.
#include "fft.h"
#include "batch.h"

namespace ml {

constexpr int radix_of(int n) { return n % 8 == 0 ? 8 : n % 4 == 0 ? 4 : n % 2 == 0 ? 2 : 3; }
constexpr int plan_radix(int n, int s) {
    for (int i = 0; i < s; ++i) n /= radix_of(n);
    return radix_of(n);
}

constexpr int NT = 256;  // threads per workgroup of every FFT kernel

// One Stockham stage of radix R at span P (product of earlier radices).
template <class T, int N, int W, int R, int P, int S>
__device__ __forceinline__ void fft_stage(cx<T>* buf, const cx<T>* tw, int tid) {
    constexpr int LD = W + 1;
    constexpr int NB = N / R;
    constexpr int TOT = NB * W;
    constexpr int IT = (TOT + NT - 1) / NT;
    cx<T> u[IT][R];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        int b = tid + it * NT;
        if (TOT % NT == 0 || b < TOT) {
            int w = b % W, i = b / W;
#pragma unroll
            for (int r = 0; r < R; ++r) u[it][r] = buf[(i + r * NB) * LD + w];
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        int b = tid + it * NT;
        if (TOT % NT == 0 || b < TOT) {
            int w = b % W, i = b / W;
            int k = i % P;
            if constexpr (P > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    cx<T> t = tw[r * k * (N / (P * R))];
                    if constexpr (S < 0) t.im = -t.im;
                    u[it][r] = cmul(u[it][r], t);
                }
            }
            dft<R, S>(u[it]);
            int j = (i - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) buf[(j + r * P) * LD + w] = u[it][r];
        }
    }
    __syncthreads();
}

template <class T, int N, int W, int S, int STAGE = 0, int P = 1>
__device__ __forceinline__ void fft_lds(cx<T>* buf, const cx<T>* tw, int tid) {
    if constexpr (P < N) {
        constexpr int R = plan_radix(N, STAGE);
        fft_stage<T, N, W, R, P, S>(buf, tw, tid);
        fft_lds<T, N, W, S, STAGE + 1, P * R>(buf, tw, tid);
    }
}

// A table of N twiddles, fetched into registers as a kernel's first loads
// and stored to LDS once its data loads are issued: loads complete in issue
// order, so the store waits for the table alone and no round trip to memory
// comes before the data loads.  Slots past N repeat the last entry.
template <class T, int N, int NTT = NT>
struct TwFetch {
    static constexpr int IT = (N + NTT - 1) / NTT;
    cx<T> v[IT];
    __device__ __forceinline__ void fetch(const cx<T>* tw, int tid) {
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            int t = tid + it * NTT;
            v[it] = tw[t < N ? t : N - 1];
        }
    }
    __device__ __forceinline__ void store(cx<T>* tw_s, int tid) const {
        issue_fence();
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            int t = tid + it * NTT;
            if (N % NTT == 0 || t < N) tw_s[t] = v[it];
        }
    }
};

// ---------------------------------------------------------------------------
// Register-resident variant for the strided passes.  Each thread keeps the
// E = W*N/NT values of its butterflies in registers across a stage; LDS is
// used only to exchange values between stages.  The first stage reads its
// inputs straight from global memory and the last stage writes its outputs
// straight back: both touch element (w, i + r*N/R), which is contiguous
// across the W pencils of a row.  Requires (N/R)*W % NT == 0 for every stage.
// ---------------------------------------------------------------------------
constexpr int num_stages(int n) {
    int c = 0;
    while (n > 1) { n /= radix_of(n); ++c; }
    return c;
}
constexpr int span_before(int n, int s) {  // product of the first s radices
    int p = 1;
    for (int i = 0; i < s; ++i) { int r = radix_of(n); p *= r; n /= r; }
    return p;
}
template <int N, int W, int NTT = NT> constexpr bool reg_path_ok() {
    int n = N;
    while (n > 1) {
        int r = radix_of(n);
        if (((N / r) * W) % NTT != 0) return false;
        n /= r;
    }
    return true;
}

template <class T, int N, int W, int R, int P, int S, int NTT = NT>
__device__ __forceinline__ void reg_compute(cx<T>* v, const cx<T>* tw, int tid) {
    constexpr int IT = (N / R) * W / NTT;
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        int i = (tid + it * NTT) / W;
        int k = i % P;
        if constexpr (P > 1) {
#pragma unroll
            for (int r = 1; r < R; ++r) {
                cx<T> t = tw[r * k * (N / (P * R))];
                if constexpr (S < 0) t.im = -t.im;
                v[it * R + r] = cmul(v[it * R + r], t);
            }
        }
        dft<R, S>(v + it * R);
    }
}

template <class T, int N, int W, int R, int P, int NTT = NT>
__device__ __forceinline__ void reg_write_lds(const cx<T>* v, cx<T>* buf, int tid) {
    constexpr int IT = (N / R) * W / NTT;
    constexpr int LD = W + 1;
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        int b = tid + it * NTT, w = b % W, i = b / W;
        int k = i % P;
        int j = (i - k) * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) buf[(j + r * P) * LD + w] = v[it * R + r];
    }
}

template <class T, int N, int W, int R, int NTT = NT>
__device__ __forceinline__ void reg_read_lds(cx<T>* v, const cx<T>* buf, int tid) {
    constexpr int IT = (N / R) * W / NTT;
    constexpr int LD = W + 1;
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        int b = tid + it * NTT, w = b % W, i = b / W;
#pragma unroll
        for (int r = 0; r < R; ++r) v[it * R + r] = buf[(i + r * (N / R)) * LD + w];
    }
}

// Element (w, n) of the tile for register slot (it, r) of a radix-R stage in
// its input pattern n = i + r*N/R.
template <int N, int W, int R, int NTT = NT>
__device__ __forceinline__ void slot_pos(int tid, int it, int r, int& w, int& n) {
    int b = tid + it * NTT;
    w = b % W;
    n = b / W + r * (N / R);
}

// Stages STAGE.. of a transform whose stage STAGE-1 outputs sit in v.
template <class T, int N, int W, int S, int STAGE, int NTT = NT>
__device__ __forceinline__ void reg_chain(cx<T>* v, cx<T>* buf, const cx<T>* tw, int tid) {
    if constexpr (STAGE < num_stages(N)) {
        constexpr int RP = plan_radix(N, STAGE - 1), PP = span_before(N, STAGE - 1);
        constexpr int R = plan_radix(N, STAGE), P = span_before(N, STAGE);
        reg_write_lds<T, N, W, RP, PP, NTT>(v, buf, tid);
        __syncthreads();
        reg_read_lds<T, N, W, R, NTT>(v, buf, tid);
        __syncthreads();
        reg_compute<T, N, W, R, P, S, NTT>(v, tw, tid);
        reg_chain<T, N, W, S, STAGE + 1, NTT>(v, buf, tw, tid);
    }
}

// ---------------------------------------------------------------------------
// pass 1: r2c along the contiguous axis.  H = Nm/2.
// `io` holds nrows rows of 2H reals on input and H complex on output.
// ---------------------------------------------------------------------------
// When hm.halo is set, the rows are a freshly painted density whose paint
// boxes' upper shells have not been merged yet: once the rows are in LDS the
// cells owed a shell add it (the same sum, in the same order, as the merge
// kernel of the paint), so the transform sees the merged density.
// Workgroup renumbering of the contiguous-axis passes: with 8 float rows
// per workgroup (meshes above 512) each XCD walks a contiguous run of row
// groups, which measured faster there; with 16 rows the hardware order
// measured faster.  A bijection of [0, nb) whenever nb % 8 == 0.
template <class T, int W>
__device__ __forceinline__ unsigned row_wg(unsigned b, unsigned nb) {
    if constexpr (sizeof(T) != 4 || W != 8) {
        return b;
    } else {
        if (nb % 8) return b;
        return (b % 8) * (nb / 8) + b / 8;
    }
}

template <class T, int H, int W>
__device__ __forceinline__ void r2c_rows_body(T* io, cx<T>* nyq, const cx<T>* tw_h,
                                                 const cx<T>* tw_post, HaloMerge<T> hm) {
    __shared__ cx<T> buf[H * (W + 1)];
    __shared__ cx<T> tws[H];
    __shared__ cx<T> twp[H / 2 + 1];
    constexpr int LD = W + 1;
    const int tid = threadIdx.x;
    const size_t r0 = (size_t)row_wg<T, W>(blockIdx.x, gridDim.x) * W;
    TwFetch<T, H> twr;
    TwFetch<T, H / 2 + 1> twq;
    twr.fetch(tw_h, tid);
    twq.fetch(tw_post, tid);
    const cx<T>* in = reinterpret_cast<const cx<T>*>(io) + r0 * H;
    {
        constexpr int IT = (W * H + NT - 1) / NT;
        cx<T> v[IT];
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            int f = tid + it * NT;
            if ((W * H) % NT == 0 || f < W * H) v[it] = in[f];  // rows are contiguous
        }
        twr.store(tws, tid);
        twq.store(twp, tid);
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            int f = tid + it * NT;
            if ((W * H) % NT == 0 || f < W * H) buf[(f % H) * LD + f / H] = v[it];
        }
    }
    __syncthreads();
    // rows r0 .. r0 + W - 1 share X (2H is a multiple of W)
    if (hm.halo) merge_rows<T, H, W, NT>(hm, buf, (int)(r0 / (2 * H)), (int)(r0 % (2 * H)), tid);
    fft_lds<T, H, W, 1>(buf, tws, tid);
    cx<T>* out = reinterpret_cast<cx<T>*>(io) + r0 * H;
    constexpr int HK = H / 2 + 1;
    for (int f = tid; f < W * HK; f += NT) {
        int w = f / HK, k = f % HK;
        cx<T> a = buf[k * LD + w];
        cx<T> b = conj(buf[((H - k) % H) * LD + w]);
        cx<T> ze = scale(a + b, T(0.5));
        cx<T> d = scale(a - b, T(0.5));
        cx<T> zo = {d.im, -d.re};  // (a - b) / (2i)
        cx<T> tzo = cmul(twp[k], zo);
        cx<T> xk = ze + tzo;
        cx<T> xm = conj(ze - tzo);
        if (k == 0) {
            out[(size_t)w * H] = xk;
            nyq[r0 + w] = xm;
        } else {
            out[(size_t)w * H + k] = xk;
            if (H - k != k) out[(size_t)w * H + (H - k)] = xm;
        }
    }
}

template <class T, int H, int W>
__global__ __launch_bounds__(NT) void k_r2c_rows(T* io, cx<T>* nyq, const cx<T>* tw_h,
                                                 const cx<T>* tw_post, HaloMerge<T> hm) {
    r2c_rows_body<T, H, W>(io, nyq, tw_h, tw_post, hm);
}
template <class T, int H, int W>
__global__ __launch_bounds__(NT) void k_r2c_rows_b(const R2cArgs<T>* __restrict__ tab) {
    const R2cArgs<T> a = tab[blockIdx.y];
    if (!a.on) return;
    r2c_rows_body<T, H, W>(a.io, a.nyq, a.tw_h, a.tw_post, a.hm);
}

// ---------------------------------------------------------------------------
// pass 5: c2r along the contiguous axis (unnormalised inverse).
// ---------------------------------------------------------------------------
// With mul_k2 the spectrum is multiplied by n2 = k2 as it is loaded (zero on
// the Nyquist plane k2 = N/2): the axis-2 gradient component of the fused
// axis-0 pass.
template <class T, int H, int W>
__device__ __forceinline__ void c2r_rows_body(T* io, const cx<T>* nyq, const cx<T>* tw_h,
                                                 const cx<T>* tw_post, int mul_k2) {
    __shared__ cx<T> buf[H * (W + 1)];
    __shared__ cx<T> tws[H];
    constexpr int LD = W + 1;
    const int tid = threadIdx.x;
    const size_t r0 = (size_t)row_wg<T, W>(blockIdx.x, gridDim.x) * W;
    TwFetch<T, H> twr;
    twr.fetch(tw_h, tid);
    const cx<T>* in = reinterpret_cast<const cx<T>*>(io) + r0 * H;
    constexpr int HK = H / 2 + 1;
    constexpr int ITK = (W * HK + NT - 1) / NT;
    cx<T> xkv[ITK], xmv[ITK], tpv[ITK];
    // every load unconditional (slots past the end repeat the last one and
    // are not used), so that all are in flight together
#pragma unroll
    for (int it = 0; it < ITK; ++it) {
        int f = tid + it * NT;
        f = f < W * HK ? f : W * HK - 1;
        int w = f / HK, k = f % HK;
        xkv[it] = in[(size_t)w * H + k];
        xmv[it] = k == 0 ? nyq[r0 + w] : in[(size_t)w * H + (H - k)];
        tpv[it] = tw_post[k];
    }
    twr.store(tws, tid);
#pragma unroll
    for (int it = 0; it < ITK; ++it) {
        int f = tid + it * NT;
        if (f >= W * HK) continue;
        int w = f / HK, k = f % HK;
        cx<T> xk = xkv[it], xm = xmv[it];
        if (mul_k2) {  // after all loads are in flight
            xk = scale(xk, T(k));
            xm = scale(xm, k == 0 ? T(0) : T(H - k));
        }
        if (k == 0) {
            xk.im = T(0);
            xm.im = T(0);
        }
        cx<T> ze = xk + conj(xm);
        cx<T> d = xk - conj(xm);
        cx<T> tp = conj(tpv[it]);  // exp(+2 pi i k / Nm)
        cx<T> q = cmul(d, tp);
        cx<T> iq = {-q.im, q.re};
        buf[k * LD + w] = ze + iq;
        if (k != 0 && H - k != k) {
            cx<T> iqc = {q.im, q.re};  // i * conj(q)
            buf[(H - k) * LD + w] = conj(ze) + iqc;
        }
    }
    __syncthreads();
    fft_lds<T, H, W, -1>(buf, tws, tid);
    cx<T>* out = reinterpret_cast<cx<T>*>(io) + r0 * H;
#pragma unroll
    for (int it = 0; it < (W * H + NT - 1) / NT; ++it) {
        int f = tid + it * NT;
        if ((W * H) % NT == 0 || f < W * H) out[f] = buf[(f % H) * LD + f / H];
    }
}

template <class T, int H, int W>
__global__ __launch_bounds__(NT) void k_c2r_rows(T* io, const cx<T>* nyq, const cx<T>* tw_h,
                                                 const cx<T>* tw_post, int mul_k2) {
    c2r_rows_body<T, H, W>(io, nyq, tw_h, tw_post, mul_k2);
}
template <class T, int H, int W>
__global__ __launch_bounds__(NT) void k_c2r_rows_b(const C2rArgs<T>* __restrict__ tab) {
    const C2rArgs<T> a = tab[blockIdx.y];
    if (!a.on) return;
    c2r_rows_body<T, H, W>(a.io, a.nyq, a.tw_h, a.tw_post, a.mul_k2);
}

// ---------------------------------------------------------------------------
// passes 2 and 4: c2c along a strided axis.  A "view" describes pencils of
// length N: element n of pencil w of workgroup g sits at
//   strided: base(g) + n*C + w,  base = (g / (C/W)) * N*C + (g % (C/W)) * W
//   contig : g*W*N + w*N + n
// Workgroups [0, g_main) work on view a, the rest on view b.
// ---------------------------------------------------------------------------
// Workgroups are handed to the 8 XCDs round-robin.  Renumber them so that
// each XCD walks a contiguous run of g.  When a workgroup's row segment is
// narrower than a 128-byte line (8 float pencils, meshes above 512),
// workgroups g and g + 1 share every line they touch, and such pairs then
// meet in one L2.  With full-line segments the axis-1 passes still gain
// (neighbouring pencils of one plane stay on one XCD) and the fused axis-0
// passes do not, so those keep the hardware order (ALL = false).
// A bijection of [0, nb) whenever nb % 8 == 0; the identity otherwise.
template <class T, int W, bool ALL>
__device__ __forceinline__ int view_wg(int b, int nb) {
    if constexpr (!ALL && W * sizeof(cx<T>) >= 128) {
        return b;
    } else {
        if (nb % 8) return b;
        return (b % 8) * (nb / 8) + b / 8;
    }
}

template <class T, int N, int W>
__device__ __forceinline__ long view_offset(const ViewDesc& v, int g, int w, int n) {
    if (v.contig) return ((long)g * W + w) * N + n;
    long cw = v.C / W;
    long base = (g / cw) * (long)N * v.C + (g % cw) * W;
    return base + (long)n * v.C + w;
}

template <class T, int N, int W, bool CONTIG>
__device__ __forceinline__ void view_load_t(cx<T>* buf, const ViewDesc& v, int g, int tid) {
    constexpr int LD = W + 1;
    constexpr int IT = (W * N + NT - 1) / NT;
    const cx<T>* p = reinterpret_cast<const cx<T>*>(v.ptr);
    cx<T> r[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        int f = tid + it * NT;
        if ((W * N) % NT == 0 || f < W * N) {
            int w = CONTIG ? f / N : f % W, n = CONTIG ? f % N : f / W;
            r[it] = p[view_offset<T, N, W>(v, g, w, n)];
        }
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        int f = tid + it * NT;
        if ((W * N) % NT == 0 || f < W * N) {
            int w = CONTIG ? f / N : f % W, n = CONTIG ? f % N : f / W;
            buf[n * LD + w] = r[it];
        }
    }
}

template <class T, int N, int W>
__device__ __forceinline__ void view_load(cx<T>* buf, const ViewDesc& v, int g, int tid) {
    if (v.contig) view_load_t<T, N, W, true>(buf, v, g, tid);
    else view_load_t<T, N, W, false>(buf, v, g, tid);
}

template <class T, int N, int W, bool CONTIG>
__device__ __forceinline__ void view_store_t(const cx<T>* buf, void* dst, const ViewDesc& v, int g,
                                             int tid) {
    constexpr int LD = W + 1;
    constexpr int IT = (W * N + NT - 1) / NT;
    cx<T>* p = reinterpret_cast<cx<T>*>(dst);
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        int f = tid + it * NT;
        if ((W * N) % NT == 0 || f < W * N) {
            int w = CONTIG ? f / N : f % W, n = CONTIG ? f % N : f / W;
            p[view_offset<T, N, W>(v, g, w, n)] = buf[n * LD + w];
        }
    }
}

template <class T, int N, int W>
__device__ __forceinline__ void view_store(const cx<T>* buf, void* dst, const ViewDesc& v, int g,
                                           int tid) {
    if (v.contig) view_store_t<T, N, W, true>(buf, dst, v, g, tid);
    else view_store_t<T, N, W, false>(buf, dst, v, g, tid);
}

template <class T, int N, int W, int S>
__device__ __forceinline__ void c2c_view_body(ViewDesc va, ViewDesc vb, const cx<T>* tw) {
    __shared__ cx<T> buf[N * (W + 1)];
    __shared__ cx<T> tws[N];
    const int tid = threadIdx.x;
    int g = view_wg<T, W, true>(blockIdx.x, gridDim.x);
    const ViewDesc& v = g < va.n_wg ? va : vb;
    if (g >= va.n_wg) g -= va.n_wg;
    TwFetch<T, N> twr;
    twr.fetch(tw, tid);
    if constexpr (reg_path_ok<N, W>()) {
        if (!v.contig) {
            constexpr int E = W * N / NT;
            constexpr int R0 = plan_radix(N, 0);
            constexpr int RL = plan_radix(N, num_stages(N) - 1);
            const cx<T>* src = reinterpret_cast<const cx<T>*>(v.ptr);
            cx<T> r[E];
#pragma unroll
            for (int it = 0; it < E / R0; ++it)
#pragma unroll
                for (int q = 0; q < R0; ++q) {
                    int w, n;
                    slot_pos<N, W, R0>(tid, it, q, w, n);
                    r[it * R0 + q] = src[view_offset<T, N, W>(v, g, w, n)];
                }
            twr.store(tws, tid);
            __syncthreads();  // twiddles in LDS
            reg_compute<T, N, W, R0, 1, S>(r, tws, tid);
            reg_chain<T, N, W, S, 1>(r, buf, tws, tid);
            cx<T>* dst = reinterpret_cast<cx<T>*>(v.ptr);
#pragma unroll
            for (int it = 0; it < E / RL; ++it)
#pragma unroll
                for (int q = 0; q < RL; ++q) {
                    int w, n;
                    slot_pos<N, W, RL>(tid, it, q, w, n);
                    dst[view_offset<T, N, W>(v, g, w, n)] = r[it * RL + q];
                }
            return;
        }
    }
    view_load<T, N, W>(buf, v, g, tid);
    twr.store(tws, tid);
    __syncthreads();
    fft_lds<T, N, W, S>(buf, tws, tid);
    view_store<T, N, W>(buf, v.ptr, v, g, tid);
}

template <class T, int N, int W, int S>
__global__ __launch_bounds__(NT) void k_c2c_view(ViewDesc va, ViewDesc vb, const cx<T>* tw) {
    c2c_view_body<T, N, W, S>(va, vb, tw);
}
template <class T, int N, int W, int S>
__global__ __launch_bounds__(NT) void k_c2c_view_b(const C2cArgs<T>* __restrict__ tab) {
    const C2cArgs<T> a = tab[blockIdx.y];
    if (!a.on) return;
    c2c_view_body<T, N, W, S>(a.va, a.vb, a.tw);
}

// ---------------------------------------------------------------------------
// Inverse pass along axis 1 that produces two outputs from one input H:
//   in place:  IFFT1(n1 H)   (zero on the plane |n1| = N/2)
//   out2:      IFFT1(H)
// (the gradient components along axes 1 and 2 of the fused axis-0 pass).
// `dst2a`/`dst2b` are the bases of the second output matching va / vb.
// ---------------------------------------------------------------------------
template <class T, int N>
__device__ __forceinline__ T n1_mult(int n) {
    constexpr int HN = N / 2;
    return n == HN ? T(0) : T(n <= HN ? n : n - N);
}

template <class T, int N, int W>
__device__ __forceinline__ void c2c_view_dual_body(ViewDesc va, ViewDesc vb, cx<T>* dst2a,
                                                      cx<T>* dst2b, const cx<T>* tw) {
    __shared__ cx<T> buf[N * (W + 1)];
    __shared__ cx<T> tws[N];
    constexpr int LD = W + 1;
    const int tid = threadIdx.x;
    int g = view_wg<T, W, true>(blockIdx.x, gridDim.x);
    const bool is_a = g < va.n_wg;
    const ViewDesc& v = is_a ? va : vb;
    cx<T>* dst2 = is_a ? dst2a : dst2b;
    if (!is_a) g -= va.n_wg;
    TwFetch<T, N> twr;
    twr.fetch(tw, tid);
    if constexpr (reg_path_ok<N, W>()) {
        if (!v.contig) {
            constexpr int E = W * N / NT;
            constexpr int R0 = plan_radix(N, 0);
            constexpr int RL = plan_radix(N, num_stages(N) - 1);
            static_assert(NT % W == 0, "a thread keeps one column");
            // slot (it, q) of a radix-R pattern: row tid/W + it*(NT/W) + q*(N/R)
            // of column tid % W, i.e. a per-thread offset plus a row count
            // known at compile time times the uniform stride
            const long tbase = view_offset<T, N, W>(v, g, tid % W, tid / W);
            const long C = v.C;
            const cx<T>* src = reinterpret_cast<const cx<T>*>(v.ptr) + tbase;
            cx<T> r[E];
#pragma unroll
            for (int it = 0; it < E / R0; ++it)
#pragma unroll
                for (int q = 0; q < R0; ++q)
                    r[it * R0 + q] = src[(long)(it * (NT / W) + q * (N / R0)) * C];
            twr.store(tws, tid);
            __syncthreads();  // twiddles in LDS
            reg_compute<T, N, W, R0, 1, -1>(r, tws, tid);
            reg_chain<T, N, W, -1, 1>(r, buf, tws, tid);
            cx<T>* d2 = dst2 + tbase;
#pragma unroll
            for (int it = 0; it < E / RL; ++it)
#pragma unroll
                for (int q = 0; q < RL; ++q)
                    d2[(long)(it * (NT / W) + q * (N / RL)) * C] = r[it * RL + q];
            // reload H (this workgroup's pencils, still in L2) scaled by n1
#pragma unroll
            for (int it = 0; it < E / R0; ++it)
#pragma unroll
                for (int q = 0; q < R0; ++q) {
                    const int n = tid / W + it * (NT / W) + q * (N / R0);
                    r[it * R0 + q] =
                        scale(src[(long)(it * (NT / W) + q * (N / R0)) * C], n1_mult<T, N>(n));
                }
            __syncthreads();  // the first transform is done with buf
            reg_compute<T, N, W, R0, 1, -1>(r, tws, tid);
            reg_chain<T, N, W, -1, 1>(r, buf, tws, tid);
            cx<T>* d1 = reinterpret_cast<cx<T>*>(v.ptr) + tbase;
#pragma unroll
            for (int it = 0; it < E / RL; ++it)
#pragma unroll
                for (int q = 0; q < RL; ++q)
                    d1[(long)(it * (NT / W) + q * (N / RL)) * C] = r[it * RL + q];
            return;
        }
    }
    // LDS path: transform H, store it to out2; reload H scaled by n1,
    // transform, store in place
    view_load<T, N, W>(buf, v, g, tid);
    twr.store(tws, tid);
    __syncthreads();
    fft_lds<T, N, W, -1>(buf, tws, tid);
    view_store<T, N, W>(buf, dst2, v, g, tid);
    __syncthreads();
    view_load<T, N, W>(buf, v, g, tid);
    __syncthreads();
    for (int f = tid; f < N * W; f += NT) {
        int n = f / W, w = f % W;
        buf[n * LD + w] = scale(buf[n * LD + w], n1_mult<T, N>(n));
    }
    __syncthreads();
    fft_lds<T, N, W, -1>(buf, tws, tid);
    view_store<T, N, W>(buf, v.ptr, v, g, tid);
}

template <class T, int N, int W>
__global__ __launch_bounds__(NT) void k_c2c_view_dual(ViewDesc va, ViewDesc vb, cx<T>* dst2a,
                                                      cx<T>* dst2b, const cx<T>* tw) {
    c2c_view_dual_body<T, N, W>(va, vb, dst2a, dst2b, tw);
}
template <class T, int N, int W>
__global__ __launch_bounds__(NT) void k_c2c_view_dual_b(const DualArgs<T>* __restrict__ tab) {
    const DualArgs<T> a = tab[blockIdx.y];
    if (!a.on) return;
    c2c_view_dual_body<T, N, W>(a.va, a.vb, a.dst2a, a.dst2b, a.tw);
}

// ---------------------------------------------------------------------------
// pass 3: fused outer-axis pass.  Forward FFT of W pencils along axis 0,
// h = i G[n0^2+n1^2+n2^2] X, then two inverse FFTs along axis 0:
//   out0 = IFFT0(n0 h)  (zero on the plane |n0| = N/2)
//   out1 = IFFT0(h).
// The gradient components along axes 1 and 2 are n1 and n2 times h, and n1,
// n2 are constant along axis 0, so both follow from out1: the axis-1 pass
// multiplies by n1 (fft_c2c_axis1_dual), the axis-2 pass by n2
// (fft_c2r_rows with mul_k2).  The view's column c maps to (k1, k2) =
// (c / (N/2), c % (N/2)) on main, (c, N/2) on nyq.  out[j] are the bases of
// the two spectra (main or nyq part, matching va or vb); out[0] may equal
// the input.
// ---------------------------------------------------------------------------
// With 512 threads the bound asks for 4 waves per SIMD, i.e. two workgroups
// per CU, so that one workgroup's loads and stores overlap the other's
// transforms.
template <class T, int N, int W, int NTG>
__device__ __forceinline__ void grad_x0_body(ViewDesc va, ViewDesc vb, PtrTriple outa,
                                                PtrTriple outb, const cx<T>* tw, const T* G, T gscale) {
    __shared__ cx<T> buf[N * (W + 1)];
    __shared__ cx<T> tws[N];
    constexpr int LD = W + 1;
    constexpr int HN = N / 2;
    const int tid = threadIdx.x;
    int g = view_wg<T, W, false>(blockIdx.x, gridDim.x);
    const bool is_a = g < va.n_wg;
    const ViewDesc& v = is_a ? va : vb;
    const PtrTriple& out = is_a ? outa : outb;
    if (!is_a) g -= va.n_wg;
    TwFetch<T, N, NTG> twr;
    twr.fetch(tw, tid);
    constexpr int R0 = plan_radix(N, 0);
    constexpr int RL = plan_radix(N, num_stages(N) - 1);
    constexpr int PL = span_before(N, num_stages(N) - 1);

    if constexpr (reg_path_ok<N, W, NTG>()) {
        constexpr int E = W * N / NTG;
        static_assert(NTG % W == 0, "a thread keeps one column");
        // Register slot (it, q) of a radix-R pattern holds row
        // tid / W + it * (NTG / W) + q * (N / R) of column tid % W: one
        // per-thread element offset plus a row count known at compile time
        // times the (uniform) row stride.
        const int wcol = tid % W;
        const long tbase = view_offset<T, N, W>(v, g, wcol, tid / W);
        const long C = v.C;
        const cx<T>* src = reinterpret_cast<const cx<T>*>(v.ptr) + tbase;
        cx<T> spec[E];
#pragma unroll
        for (int it = 0; it < E / R0; ++it)
#pragma unroll
            for (int q = 0; q < R0; ++q)
                spec[it * R0 + q] = src[(long)(it * (NTG / W) + q * (N / R0)) * C];
        twr.store(tws, tid);
        __syncthreads();
        reg_compute<T, N, W, R0, 1, 1, NTG>(spec, tws, tid);
        reg_chain<T, N, W, 1, 1, NTG>(spec, buf, tws, tid);
        if constexpr (RL != R0) {
            // bring the spectrum into the stage-0 input pattern
            reg_write_lds<T, N, W, RL, PL, NTG>(spec, buf, tid);
            __syncthreads();
            reg_read_lds<T, N, W, R0, NTG>(spec, buf, tid);
            __syncthreads();
        }
        // spec[it*R0 + q] holds k0 = tid/W + it*(NTG/W) + q*N/R0 of pencil
        // wcol; replace it by h = i G(|n|^2) spec so that component j is
        // just n_j h
        const long c = (long)g * W + wcol;
        const int k1 = is_a ? (int)(c / HN) : (int)c;
        const int k2 = is_a ? (int)(c % HN) : HN;
        const int n1 = k1 <= HN ? k1 : k1 - N;
#pragma unroll
        for (int it = 0; it < E / R0; ++it) {
#pragma unroll
            for (int q = 0; q < R0; ++q) {
                int k0 = tid / W + it * (NTG / W) + q * (N / R0);
                int n0 = k0 <= HN ? k0 : k0 - N;
                int nsq = n0 * n0 + n1 * n1 + k2 * k2;
                T gg = G ? G[nsq] : (nsq ? gscale / T(nsq) : T(0));
                cx<T> sp = spec[it * R0 + q];
                spec[it * R0 + q] = {-gg * sp.im, gg * sp.re};
            }
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            cx<T> u[E];
#pragma unroll
            for (int it = 0; it < E / R0; ++it) {
#pragma unroll
                for (int q = 0; q < R0; ++q) {
                    int k0 = tid / W + it * (NTG / W) + q * (N / R0);
                    int n0 = k0 <= HN ? k0 : k0 - N;
                    T m = j == 1 ? T(1) : (n0 == HN || n0 == -HN) ? T(0) : T(n0);
                    u[it * R0 + q] = scale(spec[it * R0 + q], m);
                }
            }
            reg_compute<T, N, W, R0, 1, -1, NTG>(u, tws, tid);
            reg_chain<T, N, W, -1, 1, NTG>(u, buf, tws, tid);
            cx<T>* dst = reinterpret_cast<cx<T>*>(out.p[j]) + tbase;
#pragma unroll
            for (int it = 0; it < E / RL; ++it)
#pragma unroll
                for (int q = 0; q < RL; ++q)
                    dst[(long)(it * (NTG / W) + q * (N / RL)) * C] = u[it * RL + q];
            __syncthreads();  // the next component reuses buf
        }
        return;
    }

    static_assert(NTG == NT || reg_path_ok<N, W, NTG>(), "LDS path needs NT threads");
    if constexpr (NTG == NT) {
    view_load<T, N, W>(buf, v, g, tid);
    twr.store(tws, tid);
    __syncthreads();
    fft_lds<T, N, W, 1>(buf, tws, tid);

    // first inverse stage: radix R0 at span 1, no twiddles
    constexpr int NB = N / R0;
    constexpr int TOT = NB * W;
    constexpr int IT = (TOT + NT - 1) / NT;
    cx<T> spec[IT][R0];
    T gv[IT][R0];
    int n0v[IT][R0];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        int b = tid + it * NT;
        if (TOT % NT == 0 || b < TOT) {
            int w = b % W, i = b / W;
            long c = (long)g * W + w;  // column within the view (a-range is 1)
            int k1, k2;
            if (is_a) { k1 = (int)(c / HN); k2 = (int)(c % HN); }
            else      { k1 = (int)c;        k2 = HN; }
            int n1 = k1 <= HN ? k1 : k1 - N;
#pragma unroll
            for (int r = 0; r < R0; ++r) {
                int k0 = i + r * NB;
                int n0 = k0 <= HN ? k0 : k0 - N;
                spec[it][r] = buf[(i + r * NB) * LD + w];
                n0v[it][r] = n0;
                int nsq = n0 * n0 + n1 * n1 + k2 * k2;
                gv[it][r] = G ? G[nsq] : (nsq ? gscale / T(nsq) : T(0));
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 2; ++j) {
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            int b = tid + it * NT;
            if (TOT % NT == 0 || b < TOT) {
                int w = b % W, i = b / W;
                cx<T> u[R0];
#pragma unroll
                for (int r = 0; r < R0; ++r) {
                    int n0 = n0v[it][r];
                    T m = j == 1 ? gv[it][r]
                                 : (n0 == HN || n0 == -HN) ? T(0) : T(n0) * gv[it][r];
                    u[r] = {-m * spec[it][r].im, m * spec[it][r].re};  // i m spec
                }
                dft<R0, -1>(u);
#pragma unroll
                for (int r = 0; r < R0; ++r) buf[(i * R0 + r) * LD + w] = u[r];
            }
        }
        __syncthreads();
        fft_lds<T, N, W, -1, 1, R0>(buf, tws, tid);
        view_store<T, N, W>(buf, out.p[j], v, g, tid);
        __syncthreads();
    }
    }
}

template <class T, int N, int W, int NTG>
__global__ __launch_bounds__(NTG, (NTG == 512 ? 4 : 1)) void k_grad_x0(
    ViewDesc va, ViewDesc vb, PtrTriple outa, PtrTriple outb, const cx<T>* tw, const T* G,
    T gscale) {
    grad_x0_body<T, N, W, NTG>(va, vb, outa, outb, tw, G, gscale);
}
template <class T, int N, int W, int NTG>
__global__ __launch_bounds__(NTG, (NTG == 512 ? 4 : 1)) void k_grad_x0_b(
    const GradArgs<T>* __restrict__ tab) {
    const GradArgs<T> a = tab[blockIdx.y];
    if (!a.on) return;
    grad_x0_body<T, N, W, NTG>(a.va, a.vb, a.outa, a.outb, a.tw, a.G, a.gscale);
}

// ---------------------------------------------------------------------------
// Transposed fused pass (adjoint of the gradient pass): forward FFT of the
// three input spectra along axis 0, combine Y = sum_j conj(i n_j G) X_j
// = -i G sum_j n_j X_j (component j zero on its Nyquist plane), inverse FFT,
// store one spectrum (may overwrite input 0).
// ---------------------------------------------------------------------------
template <class T, int N, int W>
__global__ __launch_bounds__(NT) void k_div_x0(ViewDesc va, ViewDesc vb, PtrTriple ina,
                                               PtrTriple inb, void* outa, void* outb,
                                               const cx<T>* tw, const T* G, T gscale) {
    __shared__ cx<T> buf[N * (W + 1)];
    __shared__ cx<T> tws[N];
    constexpr int LD = W + 1;
    constexpr int HN = N / 2;
    constexpr int IT = (W * N + NT - 1) / NT;
    const int tid = threadIdx.x;
    int g = view_wg<T, W, false>(blockIdx.x, gridDim.x);
    const bool is_a = g < va.n_wg;
    ViewDesc v = is_a ? va : vb;
    const PtrTriple& in = is_a ? ina : inb;
    void* out = is_a ? outa : outb;
    if (!is_a) g -= va.n_wg;
    TwFetch<T, N> twr;
    twr.fetch(tw, tid);
    cx<T> acc[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) acc[it] = {T(0), T(0)};
    for (int j = 0; j < 3; ++j) {
        v.ptr = in.p[j];
        view_load<T, N, W>(buf, v, g, tid);
        if (j == 0) twr.store(tws, tid);
        __syncthreads();
        fft_lds<T, N, W, 1>(buf, tws, tid);
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            int f = tid + it * NT;
            if ((W * N) % NT == 0 || f < W * N) {
                int n = f / W, w = f % W;
                long c = (long)g * W + w;
                int k1 = is_a ? (int)(c / HN) : (int)c;
                int k2 = is_a ? (int)(c % HN) : HN;
                int n0 = n <= HN ? n : n - N;
                int n1 = k1 <= HN ? k1 : k1 - N;
                int nj = j == 0 ? n0 : (j == 1 ? n1 : k2);
                if (nj != HN && nj != -HN) {
                    cx<T> x = buf[n * LD + w];
                    acc[it].re += T(nj) * x.re;
                    acc[it].im += T(nj) * x.im;
                }
            }
        }
        __syncthreads();
    }
    T gg[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        int f = tid + it * NT;
        f = (W * N) % NT == 0 || f < W * N ? f : W * N - 1;
        int n = f / W, w = f % W;
        long c = (long)g * W + w;
        int k1 = is_a ? (int)(c / HN) : (int)c;
        int k2 = is_a ? (int)(c % HN) : HN;
        int n0 = n <= HN ? n : n - N;
        int n1 = k1 <= HN ? k1 : k1 - N;
        int nsq = n0 * n0 + n1 * n1 + k2 * k2;
        gg[it] = nsq ? gscale / T(nsq) : T(0);
        if (G) gg[it] = G[nsq];  // uniform: the table loads issue together
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        int f = tid + it * NT;
        if ((W * N) % NT == 0 || f < W * N) {
            int n = f / W, w = f % W;
            buf[n * LD + w] = {gg[it] * acc[it].im, -gg[it] * acc[it].re};  // -i G acc
        }
    }
    __syncthreads();
    fft_lds<T, N, W, -1>(buf, tws, tid);
    view_store<T, N, W>(buf, out, v, g, tid);
}

// ---------------------------------------------------------------------------
// host-side dispatch
// ---------------------------------------------------------------------------
// Pencils per workgroup: 16 (128-byte rows) for float up to 512, 8 above
// and for double; never more than n/2 and always a divisor of n/2, so that
// a column block of the main half spectrum never straddles a row.
template <class T> constexpr int lanes_w(int n) {
    int cap = (sizeof(T) == 4 && n < 768) ? 16 : 8;
    int w = cap;
    while (w > 1 && ((n / 2) % w != 0)) w /= 2;
    return w;
}
// Rows per workgroup of the contiguous-axis passes (n*n rows, n % 16 == 0).
template <class T> constexpr int rows_w(int n) { return (sizeof(T) == 4 && n < 768) ? 16 : 8; }

#define ML_LAUNCH(kern, grid, stream, ...)                                         \
    hipLaunchKernelGGL(kern, dim3(grid), dim3(NT), 0, stream, __VA_ARGS__)

template <class T, int H>
static void r2c_rows_n(T* io, cx<T>* nyq, const cx<T>* tw_h, const cx<T>* tw_post, long nrows,
                       hipStream_t st, HaloMerge<T> hm) {
    constexpr int W = rows_w<T>(2 * H);
    ML_LAUNCH((k_r2c_rows<T, H, W>), nrows / W, st, io, nyq, tw_h, tw_post, hm);
}
template <class T, int H>
static void c2r_rows_n(T* io, const cx<T>* nyq, const cx<T>* tw_h, const cx<T>* tw_post,
                       long nrows, hipStream_t st, int mul_k2) {
    constexpr int W = rows_w<T>(2 * H);
    ML_LAUNCH((k_c2r_rows<T, H, W>), nrows / W, st, io, nyq, tw_h, tw_post, mul_k2);
}

template <class T, int N, int S>
static void c2c_axis1_n(cx<T>* main, cx<T>* nyq, const cx<T>* tw, hipStream_t st) {
    constexpr int W = lanes_w<T>(N);
    ViewDesc va{main, N / 2, 0, (int)((long)N * (N / 2) / W)};
    ViewDesc vb{nyq, 1, 1, N / W};
    ML_LAUNCH((k_c2c_view<T, N, W, S>), va.n_wg + vb.n_wg, st, va, vb, tw);
}

template <class T, int N>
static void c2c_axis1_dual_n(cx<T>* main, cx<T>* nyq, cx<T>* main2, cx<T>* nyq2, const cx<T>* tw,
                             hipStream_t st) {
    constexpr int W = lanes_w<T>(N);
    ViewDesc va{main, N / 2, 0, (int)((long)N * (N / 2) / W)};
    ViewDesc vb{nyq, 1, 1, N / W};
    ML_LAUNCH((k_c2c_view_dual<T, N, W>), va.n_wg + vb.n_wg, st, va, vb, main2, nyq2, tw);
}

template <class T, int N, int S>
static void c2c_axis0_n(cx<T>* main, cx<T>* nyq, const cx<T>* tw, hipStream_t st) {
    constexpr int W = lanes_w<T>(N);
    ViewDesc va{main, (long)N * (N / 2), 0, (int)((long)N * (N / 2) / W)};
    ViewDesc vb{nyq, N, 0, N / W};
    ML_LAUNCH((k_c2c_view<T, N, W, S>), va.n_wg + vb.n_wg, st, va, vb, tw);
}

// The fused pass holds the spectrum and one component in registers; from 512
// up it runs 512 threads per workgroup so that each thread holds half as
// many values and the CU keeps four waves per SIMD.
template <class T> constexpr int grad_nt(int n) { return (n >= 512 && sizeof(T) == 4) ? 512 : NT; }

template <class T, int N>
static void grad_axis0_n(cx<T>* main_in, cx<T>* nyq_in, PtrTriple out_main, PtrTriple out_nyq,
                         const cx<T>* tw, const T* G, T gscale, hipStream_t st) {
    constexpr int W = lanes_w<T>(N);
    constexpr int NTG = (grad_nt<T>(N) == 512 && reg_path_ok<N, W, 512>()) ? 512 : NT;
    ViewDesc va{main_in, (long)N * (N / 2), 0, (int)((long)N * (N / 2) / W)};
    ViewDesc vb{nyq_in, N, 0, N / W};
    hipLaunchKernelGGL((k_grad_x0<T, N, W, NTG>), dim3(va.n_wg + vb.n_wg), dim3(NTG), 0, st, va, vb,
                       out_main, out_nyq, tw, G, gscale);
}

template <class T, int N>
static void div_axis0_n(PtrTriple in_main, PtrTriple in_nyq, cx<T>* out_main, cx<T>* out_nyq,
                        const cx<T>* tw, const T* G, T gscale, hipStream_t st) {
    constexpr int W = lanes_w<T>(N);
    ViewDesc va{in_main.p[0], (long)N * (N / 2), 0, (int)((long)N * (N / 2) / W)};
    ViewDesc vb{in_nyq.p[0], N, 0, N / W};
    hipLaunchKernelGGL((k_div_x0<T, N, W>), dim3(va.n_wg + vb.n_wg), dim3(NT), 0, st, va, vb,
                       in_main, in_nyq, (void*)out_main, (void*)out_nyq, tw, G, gscale);
}

// Supported lengths.  float: every mesh length; double: up to 256.
#define ML_SIZES_F(X) X(16) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) X(1024)
#define ML_SIZES_D(X) X(16) X(32) X(48) X(64) X(96) X(128) X(192) X(256)

template <class T> bool fft_supported(int n) {
#define ML_CASE(v) if (n == v) return true;
    if constexpr (sizeof(T) == 4) { ML_SIZES_F(ML_CASE) }
    else { ML_SIZES_D(ML_CASE) }
#undef ML_CASE
    return false;
}

template <class T>
void fft_r2c_rows(int n, T* io, cx<T>* nyq, const cx<T>* tw_h, const cx<T>* tw_post, hipStream_t st,
                  HaloMerge<T> hm) {
    long rows = (long)n * n;
#define ML_CASE(v) if (n == v) return r2c_rows_n<T, v / 2>(io, nyq, tw_h, tw_post, rows, st, hm);
    if constexpr (sizeof(T) == 4) { ML_SIZES_F(ML_CASE) }
    else { ML_SIZES_D(ML_CASE) }
#undef ML_CASE
}

template <class T>
void fft_c2r_rows(int n, T* io, const cx<T>* nyq, const cx<T>* tw_h, const cx<T>* tw_post,
                  hipStream_t st, bool mul_k2) {
    long rows = (long)n * n;
#define ML_CASE(v) \
    if (n == v) return c2r_rows_n<T, v / 2>(io, nyq, tw_h, tw_post, rows, st, mul_k2 ? 1 : 0);
    if constexpr (sizeof(T) == 4) { ML_SIZES_F(ML_CASE) }
    else { ML_SIZES_D(ML_CASE) }
#undef ML_CASE
}

template <class T>
void fft_c2c_axis1(int n, int sign, cx<T>* main, cx<T>* nyq, const cx<T>* tw, hipStream_t st) {
#define ML_CASE(v)                                                                  \
    if (n == v) {                                                                   \
        if (sign > 0) return c2c_axis1_n<T, v, 1>(main, nyq, tw, st);               \
        return c2c_axis1_n<T, v, -1>(main, nyq, tw, st);                            \
    }
    if constexpr (sizeof(T) == 4) { ML_SIZES_F(ML_CASE) }
    else { ML_SIZES_D(ML_CASE) }
#undef ML_CASE
}

template <class T>
void fft_c2c_axis1_dual(int n, cx<T>* main, cx<T>* nyq, cx<T>* main2, cx<T>* nyq2, const cx<T>* tw,
                        hipStream_t st) {
#define ML_CASE(v) \
    if (n == v) return c2c_axis1_dual_n<T, v>(main, nyq, main2, nyq2, tw, st);
    if constexpr (sizeof(T) == 4) { ML_SIZES_F(ML_CASE) }
    else { ML_SIZES_D(ML_CASE) }
#undef ML_CASE
}

template <class T>
void fft_c2c_axis0(int n, int sign, cx<T>* main, cx<T>* nyq, const cx<T>* tw, hipStream_t st) {
#define ML_CASE(v)                                                                  \
    if (n == v) {                                                                   \
        if (sign > 0) return c2c_axis0_n<T, v, 1>(main, nyq, tw, st);               \
        return c2c_axis0_n<T, v, -1>(main, nyq, tw, st);                            \
    }
    if constexpr (sizeof(T) == 4) { ML_SIZES_F(ML_CASE) }
    else { ML_SIZES_D(ML_CASE) }
#undef ML_CASE
}

template <class T>
void fft_grad_axis0(int n, cx<T>* main_in, cx<T>* nyq_in, PtrTriple out_main, PtrTriple out_nyq,
                    const cx<T>* tw, const T* G, T gscale, hipStream_t st) {
#define ML_CASE(v) if (n == v) return grad_axis0_n<T, v>(main_in, nyq_in, out_main, out_nyq, tw, G, gscale, st);
    if constexpr (sizeof(T) == 4) { ML_SIZES_F(ML_CASE) }
    else { ML_SIZES_D(ML_CASE) }
#undef ML_CASE
}

template <class T>
void fft_div_axis0(int n, PtrTriple in_main, PtrTriple in_nyq, cx<T>* out_main, cx<T>* out_nyq,
                   const cx<T>* tw, const T* G, T gscale, hipStream_t st) {
#define ML_CASE(v) if (n == v) return div_axis0_n<T, v>(in_main, in_nyq, out_main, out_nyq, tw, G, gscale, st);
    if constexpr (sizeof(T) == 4) { ML_SIZES_F(ML_CASE) }
    else { ML_SIZES_D(ML_CASE) }
#undef ML_CASE
}

// ---- batched launches (one launch per pass over the slots of a batch) ----
template <class T>
C2cArgs<T> fft_c2c_axis1_args(int n, cx<T>* main, cx<T>* nyq, const cx<T>* tw) {
    C2cArgs<T> a{};
    const int W = lanes_w<T>(n);
    a.va = ViewDesc{main, n / 2, 0, (int)((long)n * (n / 2) / W)};
    a.vb = ViewDesc{nyq, 1, 1, n / W};
    a.tw = tw;
    a.on = 1;
    return a;
}

template <class T>
DualArgs<T> fft_c2c_axis1_dual_args(int n, cx<T>* main, cx<T>* nyq, cx<T>* main2, cx<T>* nyq2,
                                    const cx<T>* tw) {
    DualArgs<T> a{};
    const int W = lanes_w<T>(n);
    a.va = ViewDesc{main, n / 2, 0, (int)((long)n * (n / 2) / W)};
    a.vb = ViewDesc{nyq, 1, 1, n / W};
    a.dst2a = main2;
    a.dst2b = nyq2;
    a.tw = tw;
    a.on = 1;
    return a;
}

template <class T>
GradArgs<T> fft_grad_axis0_args(int n, cx<T>* main_in, cx<T>* nyq_in, PtrTriple out_main,
                                PtrTriple out_nyq, const cx<T>* tw, const T* G, T gscale) {
    GradArgs<T> a{};
    const int W = lanes_w<T>(n);
    a.va = ViewDesc{main_in, (long)n * (n / 2), 0, (int)((long)n * (n / 2) / W)};
    a.vb = ViewDesc{nyq_in, n, 0, n / W};
    a.outa = out_main;
    a.outb = out_nyq;
    a.tw = tw;
    a.G = G;
    a.gscale = gscale;
    a.on = 1;
    return a;
}

template <class T, int H>
static void r2c_rows_batch_n(const R2cArgs<T>* tab, long nrows, int slots, hipStream_t st) {
    constexpr int W = rows_w<T>(2 * H);
    hipLaunchKernelGGL((k_r2c_rows_b<T, H, W>), dim3(nrows / W, slots), dim3(NT), 0, st, tab);
}
template <class T, int H>
static void c2r_rows_batch_n(const C2rArgs<T>* tab, long nrows, int slots, hipStream_t st) {
    constexpr int W = rows_w<T>(2 * H);
    hipLaunchKernelGGL((k_c2r_rows_b<T, H, W>), dim3(nrows / W, slots), dim3(NT), 0, st, tab);
}
template <class T, int N, int S>
static void c2c_axis1_batch_n(const C2cArgs<T>* tab, int slots, hipStream_t st) {
    constexpr int W = lanes_w<T>(N);
    const int nwg = (int)((long)N * (N / 2) / W) + N / W;
    hipLaunchKernelGGL((k_c2c_view_b<T, N, W, S>), dim3(nwg, slots), dim3(NT), 0, st, tab);
}
template <class T, int N>
static void c2c_axis1_dual_batch_n(const DualArgs<T>* tab, int slots, hipStream_t st) {
    constexpr int W = lanes_w<T>(N);
    const int nwg = (int)((long)N * (N / 2) / W) + N / W;
    hipLaunchKernelGGL((k_c2c_view_dual_b<T, N, W>), dim3(nwg, slots), dim3(NT), 0, st, tab);
}
template <class T, int N>
static void grad_axis0_batch_n(const GradArgs<T>* tab, int slots, hipStream_t st) {
    constexpr int W = lanes_w<T>(N);
    constexpr int NTG = (grad_nt<T>(N) == 512 && reg_path_ok<N, W, 512>()) ? 512 : NT;
    const int nwg = (int)((long)N * (N / 2) / W) + N / W;
    hipLaunchKernelGGL((k_grad_x0_b<T, N, W, NTG>), dim3(nwg, slots), dim3(NTG), 0, st, tab);
}

template <class T>
void fft_r2c_rows_batch(int n, const R2cArgs<T>* tab, int slots, hipStream_t st) {
    long rows = (long)n * n;
#define ML_CASE(v) if (n == v) return r2c_rows_batch_n<T, v / 2>(tab, rows, slots, st);
    if constexpr (sizeof(T) == 4) { ML_SIZES_F(ML_CASE) }
    else { ML_SIZES_D(ML_CASE) }
#undef ML_CASE
}

template <class T>
void fft_c2r_rows_batch(int n, const C2rArgs<T>* tab, int slots, hipStream_t st) {
    long rows = (long)n * n;
#define ML_CASE(v) if (n == v) return c2r_rows_batch_n<T, v / 2>(tab, rows, slots, st);
    if constexpr (sizeof(T) == 4) { ML_SIZES_F(ML_CASE) }
    else { ML_SIZES_D(ML_CASE) }
#undef ML_CASE
}

template <class T>
void fft_c2c_axis1_batch(int n, int sign, const C2cArgs<T>* tab, int slots, hipStream_t st) {
#define ML_CASE(v)                                                                  \
    if (n == v) {                                                                   \
        if (sign > 0) return c2c_axis1_batch_n<T, v, 1>(tab, slots, st);            \
        return c2c_axis1_batch_n<T, v, -1>(tab, slots, st);                         \
    }
    if constexpr (sizeof(T) == 4) { ML_SIZES_F(ML_CASE) }
    else { ML_SIZES_D(ML_CASE) }
#undef ML_CASE
}

template <class T>
void fft_c2c_axis1_dual_batch(int n, const DualArgs<T>* tab, int slots, hipStream_t st) {
#define ML_CASE(v) if (n == v) return c2c_axis1_dual_batch_n<T, v>(tab, slots, st);
    if constexpr (sizeof(T) == 4) { ML_SIZES_F(ML_CASE) }
    else { ML_SIZES_D(ML_CASE) }
#undef ML_CASE
}

template <class T>
void fft_grad_axis0_batch(int n, const GradArgs<T>* tab, int slots, hipStream_t st) {
#define ML_CASE(v) if (n == v) return grad_axis0_batch_n<T, v>(tab, slots, st);
    if constexpr (sizeof(T) == 4) { ML_SIZES_F(ML_CASE) }
    else { ML_SIZES_D(ML_CASE) }
#undef ML_CASE
}

#define ML_INST_BATCH(T)                                                                           \
    template C2cArgs<T> fft_c2c_axis1_args<T>(int, cx<T>*, cx<T>*, const cx<T>*);                  \
    template DualArgs<T> fft_c2c_axis1_dual_args<T>(int, cx<T>*, cx<T>*, cx<T>*, cx<T>*,           \
                                                    const cx<T>*);                                \
    template GradArgs<T> fft_grad_axis0_args<T>(int, cx<T>*, cx<T>*, PtrTriple, PtrTriple,         \
                                                const cx<T>*, const T*, T);                       \
    template void fft_r2c_rows_batch<T>(int, const R2cArgs<T>*, int, hipStream_t);                \
    template void fft_c2r_rows_batch<T>(int, const C2rArgs<T>*, int, hipStream_t);                \
    template void fft_c2c_axis1_batch<T>(int, int, const C2cArgs<T>*, int, hipStream_t);          \
    template void fft_c2c_axis1_dual_batch<T>(int, const DualArgs<T>*, int, hipStream_t);         \
    template void fft_grad_axis0_batch<T>(int, const GradArgs<T>*, int, hipStream_t);
ML_INST_BATCH(float)
ML_INST_BATCH(double)

#define ML_INST(T)                                                                                  \
    template void fft_div_axis0<T>(int, PtrTriple, PtrTriple, cx<T>*, cx<T>*, const cx<T>*,        \
                                   const T*, T, hipStream_t);                                       \
    template bool fft_supported<T>(int);                                                            \
    template void fft_r2c_rows<T>(int, T*, cx<T>*, const cx<T>*, const cx<T>*, hipStream_t,        \
                                  HaloMerge<T>);                                                  \
    template void fft_c2r_rows<T>(int, T*, const cx<T>*, const cx<T>*, const cx<T>*, hipStream_t,  \
                                  bool);                                                          \
    template void fft_c2c_axis1<T>(int, int, cx<T>*, cx<T>*, const cx<T>*, hipStream_t);           \
    template void fft_c2c_axis1_dual<T>(int, cx<T>*, cx<T>*, cx<T>*, cx<T>*, const cx<T>*,          \
                                        hipStream_t);                                             \
    template void fft_c2c_axis0<T>(int, int, cx<T>*, cx<T>*, const cx<T>*, hipStream_t);           \
    template void fft_grad_axis0<T>(int, cx<T>*, cx<T>*, PtrTriple, PtrTriple, const cx<T>*,        \
                                    const T*, T, hipStream_t);
ML_INST(float)
ML_INST(double)

}  // namespace ml
