// Internal descriptors shared by the host orchestration and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hpnfft {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kMaxM2 = 16;         // 2m <= 16  (m <= 8)
constexpr int kMaxN = 1024;        // largest oversampled grid edge
constexpr int kLdsBytes = 160 * 1024;  // gfx950 local data share per CU

// One transform of a plan (a plan over B transforms holds B of these in
// device memory).  Grid storage is C order over (l0, l1, l2), l2 fastest, with
// cell l_t stored at l_t mod n_t.
struct Xform {
    int n[3];          // oversampled grid edges n_t = sigma N_t
    int N[3];          // bandwidth
    int ntx, nty;      // tiles along dims 2 and 1
    int nslab;         // slabs along dim 0
    int pad0;
    long long M;       // points
    long long poff;    // first sorted point of this transform (packed arrays)
    long long foff;    // first frequency of this transform (packed fhat)
    long long key_off; // first entry of this transform's cell_start table
    void *grid;        // n0 n1 n2 complex
    void *tmpA;        // n0 n1 N2 complex
    void *tmpB;        // n0 N1 N2 complex
    const double *roll[3];  // 1/c_k for k = -N_t/2 .. N_t/2-1
    const void *tw[3];      // n_t twiddles exp(-2 pi i j / n_t), plan precision
};

// Work item of the spread / interpolation kernels: lines [lb, le) of one
// tile, restricted to one slab of planes along dim 0.
struct SItem {
    int xf, tile, slab, lb, le, pad0, pad1, pad2;
};

// Work item of an FFT pass: `count` pencils starting at (outer, inner0).
struct FItem {
    int xf, outer, inner0, count;
};

// Tiling shared by all transforms of a plan.
struct Tiling {
    int T;        // tile edge (cells) in dims 2 and 1
    int Zs;       // slab depth (planes) along dim 0
    int threads;  // threads per workgroup of spread / interp
};

// LDS bytes of the spread (comp = compensated float path) and interpolation.
inline size_t spread_lds_bytes(int T, int Zs, int M2, size_t real_bytes, bool comp)
{
    size_t P = (size_t)(T + M2 - 1);
    return (size_t)Zs * P * P * 2 * real_bytes * (comp ? 2 : 1) + 64;
}
inline size_t interp_lds_bytes(int T, int Zs, int M2, size_t real_bytes, int threads, bool grad)
{
    (void)threads;
    (void)grad;
    size_t P = (size_t)(T + M2 - 1);
    return (size_t)Zs * P * P * 2 * real_bytes + 64;
}

// Threads per workgroup the interpolation kernel is compiled for: float64
// windows of 2m >= 12 (and the gradient variant from 2m >= 6) need more than
// the 128 registers a 1024-thread workgroup leaves per lane.
constexpr int interp_max_threads(int real_bytes, int M2, bool grad)
{
    return (real_bytes == 8 && (M2 >= 12 || (grad && M2 >= 6))) || (grad && M2 >= 14) ? 512 : 1024;
}

// FFT pass identifiers.
enum Pass { P_ADJ0 = 0, P_ADJ1, P_ADJ2, P_FWD0, P_FWD1, P_FWD2, P_COUNT };

// ------------------------------------------------------------------------
// Kernel launchers (defined in the .hip files).
template <typename R> struct Launch;

hipError_t launch_zero(void *p, size_t bytes, hipStream_t s);
hipError_t launch_bin_count(const double *x, const float *xf32, long long M, const Xform &X,
                            int T, int m, int *counts, int *rank, int *err, hipStream_t s);
hipError_t launch_scan(int *data, long long n, int *tmp, hipStream_t s);
hipError_t launch_bin_scatter(const double *x, const float *xf32, long long M, const Xform &X,
                              int T, int m, const int *cell_start, const int *rank,
                              int *perm, int *pz, double *us, hipStream_t s);
hipError_t launch_line_cost(const Xform &X, int T, int Zs, int m, const int *cell_start,
                            int *cost, hipStream_t s);

template <typename R>
hipError_t launch_psi(const double *us, const int *pz, long long M, long long poff, const Xform &X,
                      int m, double b, double inv_peak, R *psi, R *dpsi, hipStream_t s);
template <typename R>
hipError_t launch_gather(const void *f, const int *perm, long long total, R *fs, hipStream_t s);
template <typename R>
hipError_t launch_scatter(const R *outs, const int *perm, long long total, void *f, hipStream_t s);
template <typename R>
hipError_t launch_grad_finish(const R *outs4, const void *f, const int *perm, long long total,
                              void *grad_f, void *grad_x, hipStream_t s);
template <typename R>
hipError_t launch_spread(int m, const Xform *dxf, const SItem *items, int nitems, int *queue,
                         Tiling t, const R *psi, const R *fs, const int *pz, const int *cell_start,
                         const Xform *hxf0, hipStream_t s);
template <typename R>
hipError_t launch_interp(int m, bool grad, const Xform *dxf, const SItem *items, int nitems, int *queue,
                         Tiling t, const R *psi, const R *dpsi, const int *pz, const int *cell_start,
                         R *outs, hipStream_t s);
template <typename R>
hipError_t launch_fft(int pass, const Xform *dxf, const FItem *items, int nitems, int max_n,
                      void *fhat_base, hipStream_t s);
template <typename R>
hipError_t launch_ewald(const void *S, const Xform &X, double L, double alpha, double *partials,
                        int nblocks, double *energy, void *gbar, hipStream_t s);

}  // namespace hpnfft
