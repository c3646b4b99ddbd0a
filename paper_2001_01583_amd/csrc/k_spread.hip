// Spreading (Section 3, the Spreading step of Algorithm 2) and interpolation
// (the Interpolating step of Algorithm 5) on gfx950.
//
// The paper assigns one thread per point and adds every window tap to the
// grid with an atomic operation.  Here points are sorted by z-line (fixed
// cells in dims 1 and 2, increasing cell along dim 0), and a work item is
// one tile of T x T lines restricted to a slab of Zs planes along dim 0.
//
//   * lane <-> one (dy, dx) tap row of the point's (2m)^2 rows; a wavefront
//     holds 64 rows (a row group), the (2m)^2 rows need ceil((2m)^2/64);
//   * along dim 0 every lane keeps a register window of 2m complex values,
//     slot s holding grid plane q with q = s (mod 2m).  Consecutive points
//     of a line share the lane's row, so their taps accumulate in registers;
//     a plane leaves the window (spread: one LDS add) only when the sweep
//     has passed it.  Window weights along dim 0 are stored pre-rotated per
//     point, so slot indices are compile-time constants;
//   * the LDS tile holds the slab's planes with a halo of 2m-1 cells in dims
//     1 and 2 and is flushed to the grid with one atomic add per cell;
//   * interpolation loads the tile from the grid, slides the same register
//     window (loading a plane when it enters) and reduces the (2m)^2 row
//     partials of each point across the wavefront.
//
// Work items are taken from a device queue (one atomic per item) so heavy
// tiles and uneven batches balance across the 256 compute units.
#include <algorithm>

#include "internal.h"

namespace hpnfft {

__device__ inline int wrapn(int c, int n)
{
    c %= n;
    return c < 0 ? c + n : c;
}

__device__ inline void seg_range(int U, int z0, int zs, int m, int n0, int *a, int *b)
{
    int lo = z0 - m - U;
    int hi = z0 + zs + m - 2 - U;
    *a = lo < 0 ? 0 : lo;
    *b = hi > n0 - 1 ? n0 - 1 : hi;
}

template <typename R>
__device__ inline R wave_sum(R v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Fetch the next work item index for the whole workgroup.
__device__ inline int next_item(int *queue, int *s_item)
{
    __syncthreads();
    if (threadIdx.x == 0) *s_item = atomicAdd(queue, 1);
    __syncthreads();
    return *s_item;
}

// ---------------------------------------------------------------------------
// Spread.  COMP: float path with compensated LDS sums -- every LDS add
// returns the old value, the exact rounding error of the add is recovered
// with TwoSum and accumulated in a second array.
template <typename R, int M2, bool COMP>
__global__ __launch_bounds__(1024) void k_spread(const Xform *__restrict__ xfs,
                                                 const SItem *__restrict__ items, int nitems,
                                                 int *__restrict__ queue, int T, int Zs,
                                                 const R *__restrict__ psi, const R *__restrict__ fs,
                                                 const int *__restrict__ pz,
                                                 const int *__restrict__ cell_start)
{
    constexpr int m = M2 / 2;
    constexpr int ROWS = M2 * M2;
    constexpr int NRG = (ROWS + 63) / 64;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_item;
    const int P = T + M2 - 1;
    const int plane = P * P;
    R *acc = reinterpret_cast<R *>(smem);
    R *cmp = acc + (size_t)Zs * plane * 2;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int wave = tid >> 6, lane = tid & 63, nwaves = nthr >> 6;

    for (int it = next_item(queue, &s_item); it < nitems; it = next_item(queue, &s_item)) {
        const SItem W = items[it];
        const Xform &X = xfs[W.xf];
        const int n0 = X.n[0], n1 = X.n[1], n2 = X.n[2];
        const int X0 = (W.tile % X.ntx) * T, Y0 = (W.tile / X.ntx) * T;
        const int z0 = W.slab * Zs;
        const int zs = min(Zs, n0 - z0);
        const int ry0 = W.lb / T;
        const int nrows = (W.le - 1) / T + M2 - ry0;  // LDS rows ry0 .. ry0+nrows-1
        const int nz = zs * nrows * P;

        for (int i = tid; i < nz; i += nthr) {
            int z = i / (nrows * P), rem = i - z * nrows * P;
            size_t o = ((size_t)z * plane + (size_t)(ry0 + rem / P) * P + rem % P) * 2;
            acc[o] = R(0);
            acc[o + 1] = R(0);
            if (COMP) {
                cmp[o] = R(0);
                cmp[o + 1] = R(0);
            }
        }
        __syncthreads();

        const int nl = W.le - W.lb;
        for (int task = wave; task < nl * NRG; task += nwaves) {
            const int li = W.lb + task / NRG;
            const int rg = task % NRG;
            const int ly = li / T, lx = li % T;
            if (Y0 + ly >= n1 || X0 + lx >= n2) continue;
            const int row = rg * 64 + lane;
            const bool active = row < ROWS;
            const int dy = active ? row / M2 : 0, dx = active ? row % M2 : 0;
            const size_t lrow = (size_t)(ly + dy) * P + (lx + dx);
            const int *cs = cell_start + X.key_off + ((long long)W.tile * T * T + li) * n0;

            for (int sg = -1; sg <= 1; ++sg) {
                const int U = sg * n0;
                int a, b;
                seg_range(U, z0, zs, m, n0, &a, &b);
                if (a > b) continue;
                const long long p0 = X.poff + cs[a], p1 = X.poff + cs[b + 1];
                if (p0 >= p1) continue;
                // slab-relative plane of window plane q:  q - M2 + U - z0
                const int qshift = U - z0 - M2;

                R wr[M2], wi[M2];
#pragma unroll
                for (int s = 0; s < M2; ++s) wr[s] = wi[s] = R(0);

                auto flush = [&](int s, int q) {
                    int qr = q + qshift;
                    if (active && qr >= 0 && qr < zs) {
                        size_t o = ((size_t)qr * plane + lrow) * 2;
                        if (COMP) {
                            R vr = wr[s], vi = wi[s];
                            R old = atomicAdd(&acc[o], vr);
                            R sum = old + vr, bb = sum - old;
                            atomicAdd(&cmp[o], (old - (sum - bb)) + (vr - bb));
                            old = atomicAdd(&acc[o + 1], vi);
                            sum = old + vi;
                            bb = sum - old;
                            atomicAdd(&cmp[o + 1], (old - (sum - bb)) + (vi - bb));
                        } else {
                            atomicAdd(&acc[o], wr[s]);
                            atomicAdd(&acc[o + 1], wi[s]);
                        }
                    }
                    wr[s] = R(0);
                    wi[s] = R(0);
                };

                int Bw = -1;  // window base plane (first tap plane + M2), uniform
                for (long long p = p0; p < p1; ++p) {
                    const int B = pz[p] - m + 1 + M2;
                    if (Bw >= 0 && B != Bw) {
                        const int r = Bw % M2;
#pragma unroll
                        for (int s = 0; s < M2; ++s) {
                            const int q = Bw + (s >= r ? s - r : s - r + M2);
                            if (q < B) flush(s, q);
                        }
                    }
                    Bw = B;
                    const R *ps = psi + p * (3 * M2);
                    const R w12 = active ? ps[M2 + dy] * ps[2 * M2 + dx] : R(0);
                    const R sr = fs[2 * p] * w12, si = fs[2 * p + 1] * w12;
#pragma unroll
                    for (int s = 0; s < M2; ++s) {
                        const R wz = ps[s];
                        wr[s] = fma(sr, wz, wr[s]);
                        wi[s] = fma(si, wz, wi[s]);
                    }
                }
                const int r = Bw % M2;
#pragma unroll
                for (int s = 0; s < M2; ++s) flush(s, Bw + (s >= r ? s - r : s - r + M2));
            }
        }
        __syncthreads();

        R *grid = reinterpret_cast<R *>(X.grid);
        for (int i = tid; i < nz; i += nthr) {
            int z = i / (nrows * P), rem = i - z * nrows * P;
            int y = ry0 + rem / P, xx = rem % P;
            size_t o = ((size_t)z * plane + (size_t)y * P + xx) * 2;
            R vr = acc[o], vi = acc[o + 1];
            if (COMP) {
                vr += cmp[o];
                vi += cmp[o + 1];
            }
            int gy = wrapn(Y0 + y - m + 1, n1), gx = wrapn(X0 + xx - m + 1, n2);
            size_t g = (((size_t)(z0 + z) * n1 + gy) * n2 + gx) * 2;
            if (vr != R(0)) atomicAdd(&grid[g], vr);
            if (vi != R(0)) atomicAdd(&grid[g + 1], vi);
        }
    }
}

// ---------------------------------------------------------------------------
// Interpolation.  Output per sorted point (atomically added, zero-initialised
// by the caller):  NO = 1 complex value, or with GRAD four complex values
// (value, d/dx0, d/dx1, d/dx2).
template <typename R, int M2, bool GRAD>
__global__ __launch_bounds__(interp_max_threads(sizeof(R), M2, GRAD)) void k_interp(const Xform *__restrict__ xfs,
                                                 const SItem *__restrict__ items, int nitems,
                                                 int *__restrict__ queue, int T, int Zs,
                                                 const R *__restrict__ psi, const R *__restrict__ dpsi,
                                                 const int *__restrict__ pz,
                                                 const int *__restrict__ cell_start,
                                                 R *__restrict__ outs)
{
    constexpr int m = M2 / 2;
    constexpr int ROWS = M2 * M2;
    constexpr int NRG = (ROWS + 63) / 64;
    constexpr int NO = GRAD ? 4 : 1;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_item;
    const int P = T + M2 - 1;
    const int plane = P * P;
    R *tile = reinterpret_cast<R *>(smem);
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int wave = tid >> 6, lane = tid & 63, nwaves = nthr >> 6;

    for (int it = next_item(queue, &s_item); it < nitems; it = next_item(queue, &s_item)) {
        const SItem W = items[it];
        const Xform &X = xfs[W.xf];
        const int n0 = X.n[0], n1 = X.n[1], n2 = X.n[2];
        const int X0 = (W.tile % X.ntx) * T, Y0 = (W.tile / X.ntx) * T;
        const int z0 = W.slab * Zs;
        const int zs = min(Zs, n0 - z0);
        const int ry0 = W.lb / T;
        const int nrows = (W.le - 1) / T + M2 - ry0;
        const int nz = zs * nrows * P;
        const R *grid = reinterpret_cast<const R *>(X.grid);

        for (int i = tid; i < nz; i += nthr) {
            int z = i / (nrows * P), rem = i - z * nrows * P;
            int y = ry0 + rem / P, xx = rem % P;
            int gy = wrapn(Y0 + y - m + 1, n1), gx = wrapn(X0 + xx - m + 1, n2);
            size_t g = (((size_t)(z0 + z) * n1 + gy) * n2 + gx) * 2;
            size_t o = ((size_t)z * plane + (size_t)y * P + xx) * 2;
            tile[o] = grid[g];
            tile[o + 1] = grid[g + 1];
        }
        __syncthreads();

        const int nl = W.le - W.lb;
        for (int task = wave; task < nl; task += nwaves) {
            const int li = W.lb + task;
            const int ly = li / T, lx = li % T;
            if (Y0 + ly >= n1 || X0 + lx >= n2) continue;
            const int *cs = cell_start + X.key_off + ((long long)W.tile * T * T + li) * n0;

            for (int sg = -1; sg <= 1; ++sg) {
                const int U = sg * n0;
                int a, b;
                seg_range(U, z0, zs, m, n0, &a, &b);
                if (a > b) continue;
                const long long p0 = X.poff + cs[a], p1 = X.poff + cs[b + 1];
                const int qshift = U - z0 - M2;

                for (long long c = p0; c < p1; c += 64) {
                    const long long ce = min(p1, c + 64);
                    R ores[2 * NO];
#pragma unroll
                    for (int i = 0; i < 2 * NO; ++i) ores[i] = R(0);

                    for (int rg = 0; rg < NRG; ++rg) {
                        const int row = rg * 64 + lane;
                        const bool active = row < ROWS;
                        const int dy = active ? row / M2 : 0, dx = active ? row % M2 : 0;
                        const size_t lrow = (size_t)(ly + dy) * P + (lx + dx);
                        R gr[M2], gi[M2];
#pragma unroll
                        for (int s = 0; s < M2; ++s) gr[s] = gi[s] = R(0);
                        int Bw = -1;
                        for (long long p = c; p < ce; ++p) {
                            const int B = pz[p] - m + 1 + M2;
                            if (B != Bw) {
                                const int rn = B % M2;
                                const int ro = Bw >= 0 ? Bw % M2 : 0;
#pragma unroll
                                for (int s = 0; s < M2; ++s) {
                                    const int qold = Bw + (s >= ro ? s - ro : s - ro + M2);
                                    if (Bw < 0 || qold < B) {
                                        const int qn = B + (s >= rn ? s - rn : s - rn + M2);
                                        const int qr = qn + qshift;
                                        if (active && qr >= 0 && qr < zs) {
                                            size_t o = ((size_t)qr * plane + lrow) * 2;
                                            gr[s] = tile[o];
                                            gi[s] = tile[o + 1];
                                        } else {
                                            gr[s] = R(0);
                                            gi[s] = R(0);
                                        }
                                    }
                                }
                                Bw = B;
                            }
                            const R *ps = psi + p * (3 * M2);
                            R sr = R(0), si = R(0);
#pragma unroll
                            for (int s = 0; s < M2; ++s) {
                                sr = fma(gr[s], ps[s], sr);
                                si = fma(gi[s], ps[s], si);
                            }
                            const R w1 = active ? ps[M2 + dy] : R(0);
                            const R w2 = active ? ps[2 * M2 + dx] : R(0);
                            const R w12 = w1 * w2;
                            R v[2 * NO];
                            v[0] = sr * w12;
                            v[1] = si * w12;
                            if (GRAD) {
                                const R *dp = dpsi + p * (3 * M2);
                                R dr = R(0), di = R(0);
#pragma unroll
                                for (int s = 0; s < M2; ++s) {
                                    dr = fma(gr[s], dp[s], dr);
                                    di = fma(gi[s], dp[s], di);
                                }
                                const R d1 = active ? dp[M2 + dy] * w2 : R(0);
                                const R d2 = active ? w1 * dp[2 * M2 + dx] : R(0);
                                v[2] = dr * w12;
                                v[3] = di * w12;
                                v[4] = sr * d1;
                                v[5] = si * d1;
                                v[6] = sr * d2;
                                v[7] = si * d2;
                            }
                            const int slot = (int)(p - c);
#pragma unroll
                            for (int i = 0; i < 2 * NO; ++i) {
                                R tsum = wave_sum(v[i]);
                                if (lane == slot) ores[i] += tsum;
                            }
                        }
                    }
                    if (lane < ce - c) {
                        R *dst = outs + (c + lane) * (2 * NO);
#pragma unroll
                        for (int i = 0; i < 2 * NO; ++i) atomicAdd(&dst[i], ores[i]);
                    }
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
template <typename R, int M2>
static hipError_t spread_m(const Xform *dxf, const SItem *items, int nitems, int *queue, Tiling t,
                           const R *psi, const R *fs, const int *pz, const int *cs, hipStream_t s)
{
    constexpr bool COMP = sizeof(R) == 4;
    size_t lds = spread_lds_bytes(t.T, t.Zs, M2, sizeof(R), COMP);
    auto kern = k_spread<R, M2, COMP>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    int dev = 0, cus = 256;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    int per_cu = (int)(kLdsBytes / lds);
    if (per_cu < 1) per_cu = 1;
    int grid = cus * per_cu;
    if (grid > nitems) grid = nitems;
    if (grid < 1) return hipSuccess;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(t.threads), lds, s, dxf, items, nitems, queue, t.T, t.Zs,
                       psi, fs, pz, cs);
    return hipGetLastError();
}

template <typename R, int M2, bool GRAD>
static hipError_t interp_m(const Xform *dxf, const SItem *items, int nitems, int *queue, Tiling t,
                           const R *psi, const R *dpsi, const int *pz, const int *cs, R *outs,
                           hipStream_t s)
{
    size_t lds = interp_lds_bytes(t.T, t.Zs, M2, sizeof(R), t.threads, GRAD);
    auto kern = k_interp<R, M2, GRAD>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    int dev = 0, cus = 256;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    int per_cu = (int)(kLdsBytes / lds);
    if (per_cu < 1) per_cu = 1;
    int grid = cus * per_cu;
    if (grid > nitems) grid = nitems;
    if (grid < 1) return hipSuccess;
    int threads = std::min(t.threads, interp_max_threads(sizeof(R), M2, GRAD));
    hipLaunchKernelGGL(kern, dim3(grid), dim3(threads), lds, s, dxf, items, nitems, queue, t.T, t.Zs,
                       psi, dpsi, pz, cs, outs);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_spread(int m, const Xform *dxf, const SItem *items, int nitems, int *queue, Tiling t,
                         const R *psi, const R *fs, const int *pz, const int *cell_start,
                         const Xform *hxf0, hipStream_t s)
{
    (void)hxf0;
    switch (m) {
    case 1: return spread_m<R, 2>(dxf, items, nitems, queue, t, psi, fs, pz, cell_start, s);
    case 2: return spread_m<R, 4>(dxf, items, nitems, queue, t, psi, fs, pz, cell_start, s);
    case 3: return spread_m<R, 6>(dxf, items, nitems, queue, t, psi, fs, pz, cell_start, s);
    case 4: return spread_m<R, 8>(dxf, items, nitems, queue, t, psi, fs, pz, cell_start, s);
    case 5: return spread_m<R, 10>(dxf, items, nitems, queue, t, psi, fs, pz, cell_start, s);
    case 6: return spread_m<R, 12>(dxf, items, nitems, queue, t, psi, fs, pz, cell_start, s);
    case 7: return spread_m<R, 14>(dxf, items, nitems, queue, t, psi, fs, pz, cell_start, s);
    case 8: return spread_m<R, 16>(dxf, items, nitems, queue, t, psi, fs, pz, cell_start, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename R>
hipError_t launch_interp(int m, bool grad, const Xform *dxf, const SItem *items, int nitems, int *queue,
                         Tiling t, const R *psi, const R *dpsi, const int *pz, const int *cs, R *outs,
                         hipStream_t s)
{
#define HPNFFT_INTERP_CASE(MM)                                                                     \
    case MM:                                                                                       \
        return grad ? interp_m<R, 2 * MM, true>(dxf, items, nitems, queue, t, psi, dpsi, pz, cs,  \
                                                outs, s)                                           \
                    : interp_m<R, 2 * MM, false>(dxf, items, nitems, queue, t, psi, dpsi, pz, cs, \
                                                 outs, s);
    switch (m) {
        HPNFFT_INTERP_CASE(1)
        HPNFFT_INTERP_CASE(2)
        HPNFFT_INTERP_CASE(3)
        HPNFFT_INTERP_CASE(4)
        HPNFFT_INTERP_CASE(5)
        HPNFFT_INTERP_CASE(6)
        HPNFFT_INTERP_CASE(7)
        HPNFFT_INTERP_CASE(8)
    default: return hipErrorInvalidValue;
    }
#undef HPNFFT_INTERP_CASE
}

template hipError_t launch_spread<double>(int, const Xform *, const SItem *, int, int *, Tiling,
                                          const double *, const double *, const int *, const int *,
                                          const Xform *, hipStream_t);
template hipError_t launch_spread<float>(int, const Xform *, const SItem *, int, int *, Tiling,
                                         const float *, const float *, const int *, const int *,
                                         const Xform *, hipStream_t);
template hipError_t launch_interp<double>(int, bool, const Xform *, const SItem *, int, int *, Tiling,
                                          const double *, const double *, const int *, const int *,
                                          double *, hipStream_t);
template hipError_t launch_interp<float>(int, bool, const Xform *, const SItem *, int, int *, Tiling,
                                         const float *, const float *, const int *, const int *,
                                         float *, hipStream_t);

}  // namespace hpnfft
