// Batched launches of the fused PM step: one launch per pass steps every
// slot of a batch of simulations of one shape.  Each pass reads the
// arguments of slot y (blockIdx.y) from a device array of its argument
// structs, so that the launches, captured once in a HIP graph, replay
// unchanged while the host rewrites the arrays between steps; a slot whose
// `on` is 0 returns at once.  The per-slot grid is the single-simulation
// grid (blockIdx.x), so the kernels' workgroup renumbering is unchanged.
#pragma once
#include "fft.h"
#include "particles.h"

namespace ml {

struct FillArgs {
    uint32_t* p;
    long n;
    int on;
};

struct ScanArgs {
    const uint32_t* count;
    uint32_t* start;
    uint32_t* block_sum;
    int n;
    int on;
};

template <class T> struct ScatterArgs {
    Parts<T> src, dst;
    SortBufs s;
    Geo g;
    int on;
};

template <class T> struct PaintArgs {
    Parts<T> p;
    SortBufs s;
    Geo g;
    T mass;
    T* rho;
    T* halo;
    int on;
};

template <class T> struct LensGatherArgs {
    Parts<T> p;
    SortBufs sb;
    Geo g;
    LensArgs<T> la;
    MapAdd<T> mean;
    T* kappa;
    int on;
};

template <class T> struct ReadoutArgs {
    Parts<T> p;
    SortBufs s;
    Geo g;
    const T* f0;
    const T* f1;
    const T* f2;
    T kick;
    int do_kick;
    uint32_t* status;
    ReadoutNext<T> nx;
    int on;
};

// The FFT passes' arguments, filled by the fft_*_args helpers from the
// same pointers their single-simulation launchers take.
template <class T> struct R2cArgs {
    T* io;
    cx<T>* nyq;
    const cx<T>* tw_h;
    const cx<T>* tw_post;
    HaloMerge<T> hm;
    int on;
};
template <class T> struct C2rArgs {
    T* io;
    const cx<T>* nyq;
    const cx<T>* tw_h;
    const cx<T>* tw_post;
    int mul_k2;
    int on;
};
// the main and Nyquist-plane views of a strided pass
template <class T> struct C2cArgs {
    ViewDesc va, vb;
    const cx<T>* tw;
    int on;
};
template <class T> struct DualArgs {
    ViewDesc va, vb;
    cx<T>* dst2a;
    cx<T>* dst2b;
    const cx<T>* tw;
    int on;
};
template <class T> struct GradArgs {
    ViewDesc va, vb;
    PtrTriple outa, outb;
    const cx<T>* tw;
    const T* G;
    T gscale;
    int on;
};

// Argument builders (the single-simulation launchers' view set-up).
template <class T>
C2cArgs<T> fft_c2c_axis1_args(int n, cx<T>* main, cx<T>* nyq, const cx<T>* tw);
template <class T>
DualArgs<T> fft_c2c_axis1_dual_args(int n, cx<T>* main, cx<T>* nyq, cx<T>* main2, cx<T>* nyq2,
                                    const cx<T>* tw);
template <class T>
GradArgs<T> fft_grad_axis0_args(int n, cx<T>* main_in, cx<T>* nyq_in, PtrTriple out_main,
                                PtrTriple out_nyq, const cx<T>* tw, const T* G, T gscale);

// Batched launches over `slots` argument structs at `tab` (device memory).
void launch_fill_batch(const FillArgs* tab, long n_max, int slots, hipStream_t st);
void launch_scan_batch(const ScanArgs* tab, int n, int slots, hipStream_t st);
template <class T>
void launch_scatter_batch(const ScatterArgs<T>* tab, const Geo& g, int slots, hipStream_t st);
template <class T>
void launch_paint_batch(const PaintArgs<T>* tab, const Geo& g, int slots, hipStream_t st);
template <class T> void prepare_lens_gather_batch();
template <class T>
void launch_lens_gather_batch(const LensGatherArgs<T>* tab, const LensArgs<T>& shape, int slots,
                              hipStream_t st);
template <class T>
void launch_readout_batch(const ReadoutArgs<T>* tab, const Geo& g, int slots, hipStream_t st);
template <class T>
void fft_r2c_rows_batch(int n, const R2cArgs<T>* tab, int slots, hipStream_t st);
template <class T>
void fft_c2r_rows_batch(int n, const C2rArgs<T>* tab, int slots, hipStream_t st);
template <class T>
void fft_c2c_axis1_batch(int n, int sign, const C2cArgs<T>* tab, int slots, hipStream_t st);
template <class T>
void fft_c2c_axis1_dual_batch(int n, const DualArgs<T>* tab, int slots, hipStream_t st);
template <class T>
void fft_grad_axis0_batch(int n, const GradArgs<T>* tab, int slots, hipStream_t st);

}  // namespace ml
