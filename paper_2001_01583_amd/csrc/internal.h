// Internal descriptors shared by the host orchestration and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "window.h"

namespace hpnfft {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kMaxM2 = 30;         // 2m <= 30  (m <= 15)
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
    int flat;          // leading dims that carry no coordinate (d = 3 - flat):
                       // N_t = 1, every point at cell 0, window = unit impulse
    int nbox[3];       // box method: point bins along dims 0, 1, 2 (0: line method)
    int gbox[3];       // box method: bins per output box along dims 0, 1, 2
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

// Point bins of the box method: bin i along a dim of n cells split into nb
// bins covers cells [box_lo(i), box_lo(i + 1)); box_of inverts it.  Every
// bin is at least m cells wide, so a window reaches only the bins next to its
// own; an output box is a block of gbox consecutive bins per dim.
// (products below 1024 * 1024: grid edges and bin counts are at most kMaxN)
__host__ __device__ inline int box_lo(int i, int n, int nb) { return (int)((unsigned)(i * n) / (unsigned)nb); }
__host__ __device__ inline int box_of(int c, int n, int nb) { return (int)((unsigned)((c + 1) * nb - 1) / (unsigned)n); }
__host__ __device__ inline int box_key(const int c[3], const int n[3], const int nb[3])
{
    return (box_of(c[0], n[0], nb[0]) * nb[1] + box_of(c[1], n[1], nb[1])) * nb[2] + box_of(c[2], n[2], nb[2]);
}
// Box method record header: plane c0, and (c1 << 11) | c2 (cells < 2048).
constexpr int kBoxCellBits = 11;

// Work item of an FFT pass: `count` pencils starting at (outer, inner0).
struct FItem {
    int xf, outer, inner0, count;
};

// Tiling shared by all transforms of a plan.
struct Tiling {
    int T;        // tile edge (cells) in dims 2 and 1
    int Zs;       // slab depth (planes) along dim 0
    int threads;  // threads per workgroup of spread / interp
    int cap_hint = 0;  // points per staging chunk worth reserving (0: as many as fit)
    int ring = 0;      // spread by the ring sweep (set per launch by the plan)
};

__host__ __device__ constexpr size_t align16(size_t v) { return (v + 15) & ~(size_t)15; }

// Pointers read from a descriptor in memory (the Xform fields) are generic to
// the compiler, which then emits flat memory instructions.  A flat access also
// counts against the LDS wait counter, so every LDS wait after it would wait
// for the HBM access too.  as_global restores global addressing.
template <typename T> using gptr = __attribute__((address_space(1))) T *;
template <typename T> __device__ __forceinline__ gptr<T> as_global(T *p) { return (gptr<T>)p; }
// Read-only data (not written while the kernel runs) addressed as constant
// memory: loads from wavefront-uniform addresses become scalar loads.
template <typename T> using cptr = __attribute__((address_space(4))) const T *;
template <typename T> __device__ __forceinline__ cptr<T> as_const(const T *p) { return (cptr<T>)p; }

// Record of one sorted point (16-byte aligned, contiguous per run):
//   [psi: 3 x 2m window values (dim 0 rotated, dims 1, 2 natural)]
//   [f: the point's value, complex]  [plane index c0 (int)]
//   [line offset in its block of lines (int)]  [pad]
//   [dpsi: 3 x 2m window derivatives, gradient plans only]
__host__ __device__ constexpr size_t rec_prefix(int M2, size_t R) { return align16(3 * M2 * R + 2 * R + 8); }
__host__ __device__ constexpr size_t rec_size(int M2, size_t R, bool grad)
{
    return rec_prefix(M2, R) + (grad ? align16(3 * M2 * R) : 0);
}
__host__ __device__ constexpr size_t rec_off_f(int M2, size_t R) { return 3 * M2 * R; }
__host__ __device__ constexpr size_t rec_off_pz(int M2, size_t R) { return 3 * M2 * R + 2 * R; }
__host__ __device__ constexpr size_t rec_off_xr(int M2, size_t R) { return 3 * M2 * R + 2 * R + 4; }

// Block width: z-lines (fixed cells in dims 1 and 2) are grouped in blocks of
// BW lines adjacent along dim 2, and the points of a block are sorted by
// plane as one run.  With 2m = 8 a wavefront covers the 8 x 8 tap rows of a
// line; over a block of 8 lines each lane owns two rows of the block's 8 x 15
// footprint, so the register window a lane retires per plane serves the
// points of 8 lines instead of one.  Other windows use single lines.
__host__ __device__ constexpr int block_w(int M2) { return M2 == 8 ? 8 : 1; }

// Ring sweep of the 2m = 8 spread (ring.h): tiles of kRingT x kRingT lines,
// phases of kRingZp planes, slabs of a multiple of 2m planes.  The records store the
// dim-0 weights rotated by the absolute plane (mod 2m) while the ring counts
// planes from the slab start through the periodic images, so the plan also
// requires n0 to be a multiple of 2m.
constexpr int kRingT = 8;
constexpr int kRingZp = 8;
__host__ __device__ constexpr bool ring_tiling(int M2, int T, int Zs)
{
    return M2 == 8 && T == kRingT && Zs >= M2 && Zs % M2 == 0;
}

// Coefficients of the per-tap window polynomials (see fit_window_poly).
constexpr int kPolyF32 = 10;
constexpr int kPolyF64 = 17;
constexpr int kPolyMax = 17;

// LDS layout of the spread / interpolation kernels (bytes from the start of
// the dynamic LDS block).  kind: 0 spread, 1 interpolation, 2 gradient.
//   [tile][stage: cap records][slot maps: 2 x cap ints][run_p0: 3T^2][run_soff: 3T^2+1]
//   [scan scratch: 32 ints][a 16-byte cell that is never changed]
//   [interpolation outputs: cap x 2 NO reals]
constexpr size_t kLdsLimit = 160 * 1024 - 512;

// Row pitch (cells) of the spread's LDS tile.  The tile stores real and
// imaginary parts as separate arrays of 8-byte cells (a float32 (sum,
// compensation) pair, or a float64), so the lanes of one tap row touch
// consecutive cells.  Rows are not padded: padding them onto disjoint LDS
// banks was measured slower (it costs LDS that the staged points need).
__host__ __device__ constexpr int spread_pitch(int T, int M2) { return T + M2 - 1; }
struct LdsLayout {
    size_t tile, stage, slot_p, run_p0, run_soff, sh, out, total;
    int cap;
};
__host__ __device__ inline LdsLayout lds_layout(int T, int Zs, int M2, size_t R, int kind, bool comp, int cap)
{
    LdsLayout L{};
    size_t P = (size_t)(T + M2 - 1);
    size_t st = kind == 2 ? rec_size(M2, R, true) : rec_prefix(M2, R);
    size_t nr = (size_t)3 * T * T;
    int NO = kind == 2 ? 4 : 1;
    L.tile = 0;
    L.stage = kind == 0 ? align16((size_t)Zs * P * spread_pitch(T, M2) * 16)
                        : align16((size_t)Zs * P * P * 2 * R);
    L.slot_p = L.stage + (size_t)cap * st;
    L.run_p0 = L.slot_p + (size_t)cap * 8;
    L.run_soff = L.run_p0 + nr * 4;
    L.sh = align16(L.run_soff + (nr + 1) * 4);
    L.out = L.sh + 36 * 4;
    L.total = align16(L.out + (kind ? (size_t)cap * 2 * NO * R : 0));
    L.cap = cap;
    return L;
}
// Largest chunk capacity (points) that fits the LDS; 0 if the tile alone does not.
inline LdsLayout lds_fit(int T, int Zs, int M2, size_t R, int kind, bool comp)
{
    LdsLayout lo = lds_layout(T, Zs, M2, R, kind, comp, 0);
    if (lo.total > kLdsLimit) return LdsLayout{};
    size_t st = kind == 2 ? rec_size(M2, R, true) : rec_prefix(M2, R);
    size_t per = st + 8 + (kind ? 2 * (kind == 2 ? 4 : 1) * R : 0);
    int cap = (int)((kLdsLimit - lo.total) / per);
    if (cap > 2048) cap = 2048;
    while (cap > 0 && lds_layout(T, Zs, M2, R, kind, comp, cap).total > kLdsLimit) --cap;
    if (cap < 16) return LdsLayout{};
    return lds_layout(T, Zs, M2, R, kind, comp, cap);
}

// Threads per workgroup the sweep kernels are compiled for.  A 1024-thread
// workgroup leaves 128 registers per lane.  The spread fits (float64 with a
// few spills, measured faster than 512 threads); the interpolation variants
// that hold more window values per lane (the gradient, float64 blocked
// lines) are compiled for 512.
// Windows wider than 16 cells (m > 8) hold 2m complex values per lane in the
// register window and are compiled for 256 threads (up to 512 registers).
__host__ __device__ constexpr int spread_max_threads(int, int M2) { return M2 > 16 ? 256 : 1024; }
__host__ __device__ constexpr int interp_max_threads(int real_bytes, int M2, bool grad)
{
    return M2 > 16 ? 256
                   : (grad && (real_bytes == 8 || M2 >= 12)) || (real_bytes == 8 && block_w(M2) > 1) ? 512 : 1024;
}

// FFT pass identifiers.
enum Pass { P_ADJ0 = 0, P_ADJ1, P_ADJ2, P_FWD0, P_FWD1, P_FWD2, P_COUNT };

// ------------------------------------------------------------------------
// Kernel launchers (defined in the .hip files).
template <typename R> struct Launch;

hipError_t launch_zero(void *p, size_t bytes, hipStream_t s);
hipError_t launch_copy(void *dst, const void *src, size_t bytes, int cus, hipStream_t s);
// x / xf32 hold M x (3 - flat) coordinates; xs_out (if not null) receives
// them as M x 3 with the flat dims zero.
// Box-method plans (X.nbox[0] > 0) sort by output box instead of by line.
// keys_out (if not null) receives every point's sort key.
hipError_t launch_bin_count(const double *x, const float *xf32, long long M, const Xform &X, int T, int BW,
                            int flat, int *counts, int *rank, int *err, double *xs_out, int *keys_out,
                            hipStream_t s);
hipError_t launch_scan(int *data, long long n, int *tmp, hipStream_t s);
// fixed_pos (if not null): sorted positions already in ipos (deterministic
// mode); perm and ipos are then left as they are.
template <typename R>
hipError_t launch_bin_scatter(const double *x, const float *xf32, long long M, const Xform &X, int T, int m,
                              const WindowParams &wp, const double *poly, const int *cell_start, const int *rank, int *perm,
                              int *ipos, unsigned char *rec, size_t rec_bytes, bool grad, const int *fixed_pos,
                              hipStream_t s);
template <typename R>
hipError_t launch_gather(const void *f, const int *perm, long long total, R *fs, hipStream_t s);
template <typename R>
hipError_t launch_scatter(const R *outs, const int *ipos, long long total, void *f, hipStream_t s);
template <typename R>
hipError_t launch_grad_finish(const R *outs4, const void *f, const int *ipos, long long total, int flat,
                              void *grad_f, void *grad_x, hipStream_t s);
template <typename R>
hipError_t launch_spread(int m, const Xform *dxf, const SItem *items, int nitems, int *queue,
                         Tiling t, const unsigned char *rec, size_t rec_bytes, const R *fs, const int *cell_start,
                         hipStream_t s);
template <typename R>
hipError_t launch_interp(int m, bool grad, const Xform *dxf, const SItem *items, int nitems, int *queue,
                         Tiling t, const unsigned char *rec, size_t rec_bytes, const int *cell_start,
                         R *outs, hipStream_t s);
// Interpolation by groups of single lines (lines.h), one transform per
// launch: windows of 2m = 16 cells on grids whose n0 is a multiple of 2m.  xf: the transform's device descriptor; n: its grid edges; T: the
// tile edge of the counting sort; outs: cleared, receives sums.
template <typename R>
hipError_t launch_interp_lines(int m, const Xform *xf, const int n[3], int *queue, int T, const unsigned char *rec,
                               size_t rec_bytes, const int *cs, R *outs, hipStream_t s);
// odd: some grid edge has a factor 5 or 7
template <typename R>
hipError_t launch_fft(int pass, const Xform *dxf, const FItem *items, int nitems, int max_n, bool odd,
                      void *fhat_base, hipStream_t s);
// Ions per workgroup of the real-space pair kernel (one block partial each).
constexpr int kEwaldRealTile = 256;
hipError_t launch_ewald_real(const double *r, const double *q, long long M, double L, double alpha,
                             double rcut, double *partials, double *energy, double *forces, hipStream_t s);
// Deterministic mode (k_det.hip): stable sort by bin, one wavefront per
// output box (spread) and per point (interpolation), no atomics.
size_t det_sort_bytes(long long n);
hipError_t launch_det_sort(const int *keys, long long n, int key_bits, int *keys_out, int *vals_in, int *vals_out,
                           void *tmp, size_t tmp_bytes, long long poff, int *perm, int *ipos, hipStream_t s);
template <typename R>
hipError_t launch_spread_det(int m, const Xform *dxf, const SItem *items, int nitems, int max_cells,
                             const unsigned char *rec, size_t rec_bytes, const R *fs, const int *cell_start,
                             hipStream_t s);
template <typename R>
hipError_t launch_interp_det(int m, bool grad, const Xform *dxf, int B, long long Mtot, const unsigned char *rec,
                             size_t rec_bytes, R *outs, int cus, hipStream_t s);

// Box method (k_boxes.hip): every workgroup owns one output box of the grid
// and takes every point whose window reaches it.
template <typename R>
hipError_t launch_spread_box(int m, const Xform *dxf, const SItem *items, int nitems, int *queue, int max_cells,
                             const unsigned char *rec, size_t rec_bytes, const R *fs, const int *cell_start,
                             hipStream_t s);
template <typename R>
hipError_t launch_interp_box(int m, bool grad, const Xform *dxf, const SItem *items, int nitems, int *queue,
                             int max_cells, const unsigned char *rec, size_t rec_bytes, const int *cell_start,
                             R *outs, hipStream_t s);

// Fixed-order sum of n float64 partials into *out (one workgroup).
hipError_t launch_sum_partials(const double *part, int n, double *out, hipStream_t s);
// Cell-list real-space Ewald sum (k_ewald.hip): workspace regions and launch.
struct CellsLayout {
    size_t start, scan, cell, rank, orig, orig_tmp, sorted, sorted_tmp, part, total;
};
CellsLayout cells_layout(long long M, int nc);
hipError_t launch_ewald_cells(const double *r, const double *q, long long M, double L, double alpha, double rcut,
                              int nc, unsigned char *ws, double *energy, double *forces, hipStream_t s);
template <typename R>
hipError_t launch_ewald(const void *S, const Xform &X, double L, double alpha, double *partials,
                        int nblocks, double *energy, void *gbar, hipStream_t s);

}  // namespace hpnfft
