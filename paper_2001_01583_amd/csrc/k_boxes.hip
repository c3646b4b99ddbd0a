// Box method for sparse point sets: spreading (the Spreading step of
// Algorithm 2) and interpolation (the Interpolating step of Algorithm 5) with
// every workgroup owning one output box of the oversampled grid.
//
// At a few hundredths of a point per grid cell (the batching and Ewald
// workloads) the line sweeps of sweep.h spend their time per work item, not
// per window tap: a tile with a halo of 2m - 1 cells is cleared, flushed to
// the grid with one global atomic per cell (several times the grid, since
// neighbouring tiles overlap) and each point's window is retired plane by
// plane.  Here points are binned into bins of at least m cells per edge, so a
// window reaches only the bins next to its own (with periodic images), and
// an output box is a block of bins.  A workgroup takes one box and the points
// of its bins and of the shell of bins around them, adds the taps that fall
// inside its box into LDS (float64: native LDS atomic add; float32:
// compensated (sum, error) pairs, TwoSum and a 64-bit compare-and-swap, as in
// the line sweeps), and stores the box with plain coalesced stores: every
// grid cell is written exactly once, by its owner, with no global atomics and
// no clearing of the grid beforehand.  Interpolation loads the box once and
// adds each point's partial sum over the taps inside the box to the point's
// output (one global atomic per point and box).
//
// One wavefront handles one point at a time: its lanes take the (dim 1,
// dim 2) tap rows of the window clipped to the box, each looping over the
// clipped taps along dim 0.
#include "sweep.h"

namespace hpnfft {

constexpr int kBoxThreads = 512;
constexpr int kMaxBoxRuns = 512;  // bins around a box: (gbox + 2)^3, gbox <= 6

struct BoxGeom {
    int lo[3], w[3];  // cells of the box
    int j0[3], nj[3]; // bins of the box and its shell: j0 .. j0 + nj - 1 (may wrap)
};

__device__ inline BoxGeom box_geom(const Xform &X, int box)
{
    BoxGeom g;
    int nb[3], b[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) nb[t] = (X.nbox[t] + X.gbox[t] - 1) / X.gbox[t];
    b[2] = box % nb[2];
    b[1] = (box / nb[2]) % nb[1];
    b[0] = box / (nb[2] * nb[1]);
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        const int fb = b[t] * X.gbox[t], lb = min(fb + X.gbox[t], X.nbox[t]);
        g.lo[t] = box_lo(fb, X.n[t], X.nbox[t]);
        g.w[t] = box_lo(lb, X.n[t], X.nbox[t]) - g.lo[t];
        g.j0[t] = fb - 1;
        g.nj[t] = lb - fb + 2;
    }
    return g;
}

// Run r of the box's bins: key of the bin and the shift (0 or +-n) of its
// periodic image in each dim.
__device__ inline int box_run_bin(const Xform &X, const BoxGeom &g, int r, int sh[3])
{
    const int i2 = r % g.nj[2], i1 = (r / g.nj[2]) % g.nj[1], i0 = r / (g.nj[2] * g.nj[1]);
    int j[3] = {g.j0[0] + i0, g.j0[1] + i1, g.j0[2] + i2};
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        sh[t] = 0;
        if (j[t] < 0) {
            j[t] += X.nbox[t];
            sh[t] = -X.n[t];
        } else if (j[t] >= X.nbox[t]) {
            j[t] -= X.nbox[t];
            sh[t] = X.n[t];
        }
    }
    return (j[0] * X.nbox[1] + j[1]) * X.nbox[2] + j[2];
}

// The runs (bins) around box g: first sorted point, exclusive prefix of the
// sizes, image shifts.  Returns the number of points.  Barriers: call from
// all threads.
__device__ inline int box_runs(const Xform &X, const BoxGeom &g, const int *kcs, int *run_p0, int *run_soff,
                               int *run_sh, int *sh_scan, int *nruns)
{
    const int nr = g.nj[0] * g.nj[1] * g.nj[2];
    const int tid = threadIdx.x;
    int cnt = 0;
    if (tid < nr) {
        int sh[3];
        const int key = box_run_bin(X, g, tid, sh);
        const int a = kcs[key], b = kcs[key + 1];
        run_p0[tid] = (int)(X.poff + a);
        cnt = b - a;
        run_sh[3 * tid] = sh[0];
        run_sh[3 * tid + 1] = sh[1];
        run_sh[3 * tid + 2] = sh[2];
    }
    int total;
    const int base = block_excl_scan(cnt, sh_scan, &total);
    if (tid < nr) run_soff[tid] = base;
    if (tid == 0) run_soff[nr] = total;
    __syncthreads();
    *nruns = nr;
    return total;
}

// Window of a point image clipped to the box: taps [a_t, b_t) of the 2m taps
// along each dim, first tap cell f_t.  False if the window misses the box.
struct Clip {
    int a[3], b[3], f[3];
};
__device__ inline bool clip_window(int2 head, const int sh[3], const BoxGeom &g, int m, Clip &c)
{
    const int cell[3] = {head.x, head.y >> kBoxCellBits, head.y & ((1 << kBoxCellBits) - 1)};
    bool ok = true;
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        c.f[t] = cell[t] + sh[t] - m + 1;
        c.a[t] = max(0, g.lo[t] - c.f[t]);
        c.b[t] = min(2 * m, g.lo[t] + g.w[t] - c.f[t]);
        ok &= c.a[t] < c.b[t];
    }
    return ok;
}

// Point k (0 .. S-1) of the runs: its sorted position and image shift.
__device__ inline long long box_point(int k, int nruns, const int *run_p0, const int *run_soff, const int *run_sh,
                                      int sh[3])
{
    const int r = uni(find_run(run_soff, nruns, k));
    sh[0] = uni(run_sh[3 * r]);
    sh[1] = uni(run_sh[3 * r + 1]);
    sh[2] = uni(run_sh[3 * r + 2]);
    return (long long)uni(run_p0[r]) + (k - uni(run_soff[r]));
}

// Value of v in lane l (l wave-uniform), as a lane read: the dim-0 weights of
// a point sit one per lane, so the tap loop reads them without a memory
// access.
template <typename R> __device__ inline R lane_value(R v, int l)
{
    unsigned w[Words<R>::n];
    Words<R>::split(v, w);
#pragma unroll
    for (int i = 0; i < Words<R>::n; ++i) w[i] = (unsigned)__builtin_amdgcn_readlane((int)w[i], l);
    return Words<R>::join(w);
}

// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(kBoxThreads) void k_spread_box(const Xform *__restrict__ xfs,
                                                            const SItem *__restrict__ items, int nitems,
                                                            int *__restrict__ queue, int m,
                                                            const unsigned char *__restrict__ rec, int rec_bytes,
                                                            const R *__restrict__ fs, const int *__restrict__ cs)
{
    constexpr bool COMP = sizeof(R) == 4;
    extern __shared__ uint4 smem16[];
    __shared__ int s_item;
    __shared__ int run_p0[kMaxBoxRuns], run_soff[kMaxBoxRuns + 1], run_sh[3 * kMaxBoxRuns], sh_scan[36];
    const int M2 = 2 * m;
    const int off_pz = (int)rec_off_pz(M2, sizeof(R));
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int wave = uni(tid >> 6), lane = tid & 63, nwaves = nthr >> 6;
    // real parts [cells], then imaginary parts [cells], 8-byte cells
    unsigned long long *pairs = reinterpret_cast<unsigned long long *>(smem16);
    R *acc = reinterpret_cast<R *>(smem16);
    for (int it = next_item(queue, &s_item); it < nitems; it = next_item(queue, &s_item)) {
        const SItem W = items[it];
        const Xform &X = xfs[W.xf];
        const BoxGeom g = box_geom(X, W.tile);
        const int cells = g.w[0] * g.w[1] * g.w[2];
        for (int i = tid; i < 2 * cells; i += nthr) pairs[i] = 0ull;
        int nruns;
        const int S = box_runs(X, g, cs + X.key_off, run_p0, run_soff, run_sh, sh_scan, &nruns);
        for (int k = wave; k < S; k += nwaves) {
            int sh[3];
            const long long pos = box_point(k, nruns, run_p0, run_soff, run_sh, sh);
            const unsigned char *rp = rec + pos * rec_bytes;
            const int2 hd = *reinterpret_cast<const int2 *>(rp + off_pz);
            Clip c;
            if (!clip_window(make_int2(uni(hd.x), uni(hd.y)), sh, g, m, c)) continue;
            const R *ps = reinterpret_cast<const R *>(rp);
            const R fr = fs[2 * pos], fi = fs[2 * pos + 1];
            const R w0l = lane < M2 ? ps[lane] : R(0);  // dim-0 weight of tap `lane`
            const int n2 = c.b[2] - c.a[2], rows = (c.b[1] - c.a[1]) * n2;
            for (int i = lane; i < rows; i += 64) {
                const int t1 = c.a[1] + i / n2, t2 = c.a[2] + i % n2;
                const R w12 = ps[M2 + t1] * ps[2 * M2 + t2];
                const R vr = fr * w12, vi = fi * w12;
                const int yx = (c.f[1] + t1 - g.lo[1]) * g.w[2] + (c.f[2] + t2 - g.lo[2]);
                for (int t0 = c.a[0]; t0 < c.b[0]; ++t0) {
                    const R w = lane_value(w0l, t0);
                    const int o = (c.f[0] + t0 - g.lo[0]) * g.w[1] * g.w[2] + yx;
                    if constexpr (COMP) {
                        unsigned long long *cc[2] = {&pairs[o], &pairs[o + cells]};
                        const float v[2] = {(float)(vr * w), (float)(vi * w)};
                        const bool okk[2] = {true, true};
                        lds_add_comp<2>(cc, v, okk);
                    } else {
                        atomicAdd(&acc[o], vr * w);
                        atomicAdd(&acc[o + cells], vi * w);
                    }
                }
            }
        }
        __syncthreads();
        // the box, stored once: every cell of the grid has exactly one owner
        const gptr<R> grid = as_global(reinterpret_cast<R *>(X.grid));
        for (int i = tid; i < cells; i += nthr) {
            const int z = i / (g.w[1] * g.w[2]), rr = i - z * g.w[1] * g.w[2];
            const int y = rr / g.w[2], x = rr - y * g.w[2];
            R vr, vi;
            if constexpr (COMP) {
                const unsigned long long a0 = pairs[i], a1 = pairs[i + cells];
                vr = __uint_as_float((unsigned int)a0) + __uint_as_float((unsigned int)(a0 >> 32));
                vi = __uint_as_float((unsigned int)a1) + __uint_as_float((unsigned int)(a1 >> 32));
            } else {
                vr = acc[i];
                vi = acc[i + cells];
            }
            const size_t gi = (((size_t)(g.lo[0] + z) * X.n[1] + g.lo[1] + y) * X.n[2] + g.lo[2] + x) * 2;
            grid[gi] = vr;
            grid[gi + 1] = vi;
        }
    }
    release_queue(queue);
}

// ---------------------------------------------------------------------------

template <typename R, bool GRAD>
__global__ __launch_bounds__(kBoxThreads) void k_interp_box(const Xform *__restrict__ xfs,
                                                            const SItem *__restrict__ items, int nitems,
                                                            int *__restrict__ queue, int m,
                                                            const unsigned char *__restrict__ rec, int rec_bytes,
                                                            const int *__restrict__ cs, R *__restrict__ outs)
{
    constexpr int NO = GRAD ? 4 : 1;
    extern __shared__ uint4 smem16[];
    __shared__ int s_item;
    __shared__ int run_p0[kMaxBoxRuns], run_soff[kMaxBoxRuns + 1], run_sh[3 * kMaxBoxRuns], sh_scan[36];
    const int M2 = 2 * m;
    const int off_pz = (int)rec_off_pz(M2, sizeof(R));
    const int off_d = (int)rec_prefix(M2, sizeof(R)) / (int)sizeof(R);
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int wave = uni(tid >> 6), lane = tid & 63, nwaves = nthr >> 6;
    R *tile = reinterpret_cast<R *>(smem16);  // interleaved (re, im) per cell
    for (int it = next_item(queue, &s_item); it < nitems; it = next_item(queue, &s_item)) {
        const SItem W = items[it];
        const Xform &X = xfs[W.xf];
        const BoxGeom g = box_geom(X, W.tile);
        const int cells = g.w[0] * g.w[1] * g.w[2];
        const gptr<const R> grid = as_global(reinterpret_cast<const R *>(X.grid));
        for (int i = tid; i < cells; i += nthr) {
            const int z = i / (g.w[1] * g.w[2]), rr = i - z * g.w[1] * g.w[2];
            const int y = rr / g.w[2], x = rr - y * g.w[2];
            const size_t gi = (((size_t)(g.lo[0] + z) * X.n[1] + g.lo[1] + y) * X.n[2] + g.lo[2] + x) * 2;
            tile[2 * i] = grid[gi];
            tile[2 * i + 1] = grid[gi + 1];
        }
        int nruns;
        const int S = box_runs(X, g, cs + X.key_off, run_p0, run_soff, run_sh, sh_scan, &nruns);
        for (int k = wave; k < S; k += nwaves) {
            int sh[3];
            const long long pos = box_point(k, nruns, run_p0, run_soff, run_sh, sh);
            const unsigned char *rp = rec + pos * rec_bytes;
            const int2 hd = *reinterpret_cast<const int2 *>(rp + off_pz);
            Clip c;
            if (!clip_window(make_int2(uni(hd.x), uni(hd.y)), sh, g, m, c)) continue;
            const R *ps = reinterpret_cast<const R *>(rp);
            const R *dp = ps + off_d;
            // dim-0 weight (and derivative) of tap `lane`
            const R w0l = lane < M2 ? ps[lane] : R(0);
            const R d0l = GRAD && lane < M2 ? dp[lane] : R(0);
            R v[2 * NO];
#pragma unroll
            for (int q = 0; q < 2 * NO; ++q) v[q] = R(0);
            const int n2 = c.b[2] - c.a[2], rows = (c.b[1] - c.a[1]) * n2;
            for (int i = lane; i < rows; i += 64) {
                const int t1 = c.a[1] + i / n2, t2 = c.a[2] + i % n2;
                const int yx = (c.f[1] + t1 - g.lo[1]) * g.w[2] + (c.f[2] + t2 - g.lo[2]);
                R sr = R(0), si = R(0), dr = R(0), di = R(0);
                for (int t0 = c.a[0]; t0 < c.b[0]; ++t0) {
                    const int o = ((c.f[0] + t0 - g.lo[0]) * g.w[1] * g.w[2] + yx) * 2;
                    const R gr = tile[o], gim = tile[o + 1];
                    const R w = lane_value(w0l, t0);
                    sr = fma(w, gr, sr);
                    si = fma(w, gim, si);
                    if constexpr (GRAD) {
                        const R dw = lane_value(d0l, t0);
                        dr = fma(dw, gr, dr);
                        di = fma(dw, gim, di);
                    }
                }
                const R w1 = ps[M2 + t1], w2 = ps[2 * M2 + t2];
                const R w12 = w1 * w2;
                v[0] = fma(sr, w12, v[0]);
                v[1] = fma(si, w12, v[1]);
                if constexpr (GRAD) {
                    const R d1 = dp[M2 + t1] * w2, d2 = w1 * dp[2 * M2 + t2];
                    v[2] = fma(dr, w12, v[2]);
                    v[3] = fma(di, w12, v[3]);
                    v[4] = fma(sr, d1, v[4]);
                    v[5] = fma(si, d1, v[5]);
                    v[6] = fma(sr, d2, v[6]);
                    v[7] = fma(si, d2, v[7]);
                }
            }
            if constexpr (GRAD) {
                // the eight sums through the halving steps of wave_reduce.h
                // (about 10 lane exchanges per word instead of 48): the
                // 8-lane group j ends with the sum of value bitrev3(j), which
                // its first lane adds to the output
                const R a0 = halve32(v[0], v[1]), a1 = halve32(v[2], v[3]);
                const R a2 = halve32(v[4], v[5]), a3 = halve32(v[6], v[7]);
                const R r = halve8_sum(halve16(a0, a1), halve16(a2, a3));
                if ((lane & 7) == 0) {
                    const int j = lane >> 3;
                    const int q = ((j & 1) << 2) | (j & 2) | (j >> 2);
                    atomicAdd(&outs[pos * (2 * NO) + q], r);
                }
            } else {
                // the two sums through the same steps, each value fed in four
                // times: 8-lane groups 0-3 end with the sum of v[0], groups
                // 4-7 with that of v[1]
                const R a = halve32(v[0], v[1]);
                const R b = halve16(a, a);
                const R r = halve8_sum(b, b);
                if ((lane & 31) == 0) atomicAdd(&outs[pos * 2 + (lane >> 5)], r);
            }
        }
        __syncthreads();  // the next box overwrites the tile
    }
    release_queue(queue);
}

// ---------------------------------------------------------------------------
static int box_cus()
{
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
    }
    return cus;
}

template <typename R>
hipError_t launch_spread_box(int m, const Xform *dxf, const SItem *items, int nitems, int *queue, int max_cells,
                             const unsigned char *rec, size_t rec_bytes, const R *fs, const int *cell_start,
                             hipStream_t s)
{
    if (nitems <= 0) return hipSuccess;
    const size_t lds = (size_t)max_cells * 16;
    auto kern = k_spread_box<R>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const int per_cu = std::max(1, std::min(4, (int)((160 * 1024) / (lds + 12 * 1024))));
    const int grid = std::min(box_cus() * per_cu, nitems);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kBoxThreads), lds, s, dxf, items, nitems, queue, m, rec,
                       (int)rec_bytes, fs, cell_start);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_interp_box(int m, bool grad, const Xform *dxf, const SItem *items, int nitems, int *queue,
                             int max_cells, const unsigned char *rec, size_t rec_bytes, const int *cell_start,
                             R *outs, hipStream_t s)
{
    if (nitems <= 0) return hipSuccess;
    const size_t lds = (size_t)max_cells * 2 * sizeof(R);
    auto kern = grad ? k_interp_box<R, true> : k_interp_box<R, false>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const int per_cu = std::max(1, std::min(4, (int)((160 * 1024) / (lds + 12 * 1024))));
    const int grid = std::min(box_cus() * per_cu, nitems);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kBoxThreads), lds, s, dxf, items, nitems, queue, m, rec,
                       (int)rec_bytes, cell_start, outs);
    return hipGetLastError();
}

template hipError_t launch_spread_box<double>(int, const Xform *, const SItem *, int, int *, int,
                                              const unsigned char *, size_t, const double *, const int *,
                                              hipStream_t);
template hipError_t launch_spread_box<float>(int, const Xform *, const SItem *, int, int *, int,
                                             const unsigned char *, size_t, const float *, const int *,
                                             hipStream_t);
template hipError_t launch_interp_box<double>(int, bool, const Xform *, const SItem *, int, int *, int,
                                              const unsigned char *, size_t, const int *, double *, hipStream_t);
template hipError_t launch_interp_box<float>(int, bool, const Xform *, const SItem *, int, int *, int,
                                             const unsigned char *, size_t, const int *, float *, hipStream_t);

}  // namespace hpnfft
