// Deterministic mode (plans created with HPNFFT_DETERMINISTIC): the
// Spreading and Interpolating steps (Algorithms 2 and 5) with every sum taken
// in a fixed order, so that repeated calls, and repeated set_points of the
// same points, give bitwise identical results.
//
//   * The points are sorted by (bin, input index) with a stable radix sort
//     (rocPRIM through hipCUB), instead of the counting sort's atomic ranks.
//   * Spreading: one wavefront owns one output box (the bins of the box
//     method) and adds the points of its bins and of the shell around them
//     one after the other, in sorted order.  Within a point every lane owns
//     distinct cells, so the LDS updates are plain read-modify-writes (float32:
//     the compensated (sum, error) pair, TwoSum); the box is stored once.
//   * Interpolation: one wavefront owns one point.  Its lanes take the tap
//     rows of the point's window, read the grid cells directly (L2-cached),
//     and the lane partials are summed by a fixed butterfly; the point's
//     outputs are plain stores.
// The FFT passes and the gather / scatter kernels have no atomics.
#include <hipcub/hipcub.hpp>

#include "internal.h"

namespace hpnfft {

constexpr int kDetMaxRuns = 512;

__device__ inline int det_uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

// ---------------------------------------------------------------------------
// Stable binning: sort (key, j) pairs by key, ties in input order.
__global__ void k_iota(int *__restrict__ v, long long n)
{
    const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) v[j] = (int)j;
}

// Sorted position p of transform point perm_local[p]: perm and ipos over the
// packed arrays (offset poff).
__global__ void k_perm_ipos(const int *__restrict__ perm_local, long long n, long long poff, int *__restrict__ perm,
                            int *__restrict__ ipos)
{
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int j = perm_local[p];
    perm[poff + p] = (int)(poff + j);
    ipos[poff + j] = (int)(poff + p);
}

size_t det_sort_bytes(long long n)
{
    size_t bytes = 0;
    // (a size query: it launches nothing; on failure the sort itself reports)
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, (const int *)nullptr, (int *)nullptr,
                                             (const int *)nullptr, (int *)nullptr, (int)n, 0, 31);
    return bytes;
}

hipError_t launch_det_sort(const int *keys, long long n, int key_bits, int *keys_out, int *vals_in, int *vals_out,
                           void *tmp, size_t tmp_bytes, long long poff, int *perm, int *ipos, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const unsigned nb = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_iota, dim3(nb), dim3(256), 0, s, vals_in, n);
    size_t bytes = tmp_bytes;
    hipError_t e = hipcub::DeviceRadixSort::SortPairs(tmp, bytes, keys, keys_out, vals_in, vals_out, (int)n, 0,
                                                      key_bits, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_perm_ipos, dim3(nb), dim3(256), 0, s, vals_out, n, poff, perm, ipos);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
struct DetBox {
    int lo[3], w[3], j0[3], nj[3];
};

__device__ inline DetBox det_box(const Xform &X, int box)
{
    DetBox g;
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

template <typename R>
__global__ __launch_bounds__(64) void k_spread_det(const Xform *__restrict__ xfs, const SItem *__restrict__ items,
                                                   int m, const unsigned char *__restrict__ rec, int rec_bytes,
                                                   const R *__restrict__ fs, const int *__restrict__ cs)
{
    constexpr bool COMP = sizeof(R) == 4;
    extern __shared__ uint4 smem16[];
    __shared__ int run_p0[kDetMaxRuns], run_soff[kDetMaxRuns + 1], run_sh[3 * kDetMaxRuns];
    const int lane = threadIdx.x, M2 = 2 * m;
    const int off_pz = (int)rec_off_pz(M2, sizeof(R));
    const SItem W = items[blockIdx.x];
    const Xform &X = xfs[W.xf];
    const DetBox g = det_box(X, W.tile);
    const int cells = g.w[0] * g.w[1] * g.w[2];
    R *acc = reinterpret_cast<R *>(smem16);        // float64: re [cells], im [cells]
    float *pr = reinterpret_cast<float *>(smem16);  // float32: (sum, err) pairs, re then im
    for (int i = lane; i < 2 * cells * (COMP ? 2 : 1); i += 64) {
        if constexpr (COMP) pr[i] = 0.f;
        else acc[i] = R(0);
    }
    // runs: the bins of the box and its shell, in a fixed order
    const int *kcs = cs + X.key_off;
    const int nr = g.nj[0] * g.nj[1] * g.nj[2];
    int carry = 0;
    for (int r0 = 0; r0 < nr; r0 += 64) {
        const int r = r0 + lane;
        int cnt = 0;
        if (r < nr) {
            const int i2 = r % g.nj[2], i1 = (r / g.nj[2]) % g.nj[1], i0 = r / (g.nj[2] * g.nj[1]);
            int j[3] = {g.j0[0] + i0, g.j0[1] + i1, g.j0[2] + i2}, sh[3];
#pragma unroll
            for (int t = 0; t < 3; ++t) {
                sh[t] = 0;
                if (j[t] < 0) { j[t] += X.nbox[t]; sh[t] = -X.n[t]; }
                else if (j[t] >= X.nbox[t]) { j[t] -= X.nbox[t]; sh[t] = X.n[t]; }
            }
            const int key = (j[0] * X.nbox[1] + j[1]) * X.nbox[2] + j[2];
            const int a = kcs[key];
            cnt = kcs[key + 1] - a;
            run_p0[r] = (int)(X.poff + a);
            run_sh[3 * r] = sh[0];
            run_sh[3 * r + 1] = sh[1];
            run_sh[3 * r + 2] = sh[2];
        }
        int incl = cnt;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(incl, o, 64);
            if (lane >= o) incl += y;
        }
        if (r < nr) run_soff[r] = carry + incl - cnt;
        carry += __shfl(incl, 63, 64);
    }
    if (lane == 0) run_soff[nr] = carry;
    __syncthreads();
    // points in sorted order, one at a time
    int r = 0;
    for (int k = 0; k < carry; ++k) {
        while (det_uni(run_soff[r + 1]) <= k) ++r;
        const long long pos = (long long)det_uni(run_p0[r]) + (k - det_uni(run_soff[r]));
        const unsigned char *rp = rec + pos * rec_bytes;
        const int2 hd = *reinterpret_cast<const int2 *>(rp + off_pz);
        const int cell[3] = {det_uni(hd.x), det_uni(hd.y) >> kBoxCellBits, det_uni(hd.y) & ((1 << kBoxCellBits) - 1)};
        int a[3], b[3], f[3];
        bool ok = true;
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            f[t] = cell[t] + det_uni(run_sh[3 * r + t]) - m + 1;
            a[t] = max(0, g.lo[t] - f[t]);
            b[t] = min(M2, g.lo[t] + g.w[t] - f[t]);
            ok &= a[t] < b[t];
        }
        if (!ok) continue;
        const R *ps = reinterpret_cast<const R *>(rp);
        const R fr = fs[2 * pos], fi = fs[2 * pos + 1];
        const int n2 = b[2] - a[2], rows = (b[1] - a[1]) * n2;
        for (int i = lane; i < rows; i += 64) {
            const int t1 = a[1] + i / n2, t2 = a[2] + i % n2;
            const R w12 = ps[M2 + t1] * ps[2 * M2 + t2];
            const R vr = fr * w12, vi = fi * w12;
            const int yx = (f[1] + t1 - g.lo[1]) * g.w[2] + (f[2] + t2 - g.lo[2]);
            for (int t0 = a[0]; t0 < b[0]; ++t0) {
                const R w = ps[t0];
                const int o = (f[0] + t0 - g.lo[0]) * g.w[1] * g.w[2] + yx;
                if constexpr (COMP) {
                    // TwoSum into the (sum, error) pair of the cell (its only writer)
                    const float add[2] = {(float)(vr * w), (float)(vi * w)};
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        float *q = pr + 2 * (o + c * cells);
                        const float sm = q[0], t = sm + add[c], bp = t - sm;
                        const float e = (sm - (t - bp)) + (add[c] - bp);
                        q[0] = t;
                        q[1] += e;
                    }
                } else {
                    acc[o] += vr * w;
                    acc[o + cells] += vi * w;
                }
            }
        }
    }
    __syncthreads();
    R *grid = reinterpret_cast<R *>(X.grid);
    for (int i = lane; i < cells; i += 64) {
        const int z = i / (g.w[1] * g.w[2]), rr = i - z * g.w[1] * g.w[2];
        const int y = rr / g.w[2], x = rr - y * g.w[2];
        R vr, vi;
        if constexpr (COMP) {
            vr = pr[2 * i] + pr[2 * i + 1];
            vi = pr[2 * (i + cells)] + pr[2 * (i + cells) + 1];
        } else {
            vr = acc[i];
            vi = acc[i + cells];
        }
        const size_t gi = (((size_t)(g.lo[0] + z) * X.n[1] + g.lo[1] + y) * X.n[2] + g.lo[2] + x) * 2;
        grid[gi] = vr;
        grid[gi + 1] = vi;
    }
}

// ---------------------------------------------------------------------------
template <typename R> __device__ inline R det_wave_sum(R v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <typename R, bool GRAD>
__global__ __launch_bounds__(256) void k_interp_det(const Xform *__restrict__ xfs, int B, long long Mtot, int m,
                                                    const unsigned char *__restrict__ rec, int rec_bytes,
                                                    R *__restrict__ outs)
{
    constexpr int NO = GRAD ? 4 : 1;
    const int lane = threadIdx.x & 63, M2 = 2 * m;
    const int off_pz = (int)rec_off_pz(M2, sizeof(R));
    const int off_d = (int)rec_prefix(M2, sizeof(R)) / (int)sizeof(R);
    const long long wid = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const long long nw = ((long long)gridDim.x * blockDim.x) >> 6;
    for (long long pos = wid; pos < Mtot; pos += nw) {
        // the transform of sorted point pos (packed in order)
        int lo = 0, hi = B;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (xfs[mid].poff <= pos) lo = mid;
            else hi = mid;
        }
        const Xform &X = xfs[lo];
        const R *grid = reinterpret_cast<const R *>(X.grid);
        const unsigned char *rp = rec + pos * rec_bytes;
        const int2 hd = *reinterpret_cast<const int2 *>(rp + off_pz);
        const int c0 = hd.x, c1 = hd.y >> kBoxCellBits, c2 = hd.y & ((1 << kBoxCellBits) - 1);
        const R *ps = reinterpret_cast<const R *>(rp);
        const R *dp = ps + off_d;
        R v[2 * NO];
#pragma unroll
        for (int q = 0; q < 2 * NO; ++q) v[q] = R(0);
        for (int i = lane; i < M2 * M2; i += 64) {
            const int t1 = i / M2, t2 = i % M2;
            int l1 = c1 - m + 1 + t1, l2 = c2 - m + 1 + t2;
            l1 += l1 < 0 ? X.n[1] : (l1 >= X.n[1] ? -X.n[1] : 0);
            l2 += l2 < 0 ? X.n[2] : (l2 >= X.n[2] ? -X.n[2] : 0);
            R sr = R(0), si = R(0), dr = R(0), di = R(0);
            for (int t0 = 0; t0 < M2; ++t0) {
                int l0 = c0 - m + 1 + t0;
                l0 += l0 < 0 ? X.n[0] : (l0 >= X.n[0] ? -X.n[0] : 0);
                const size_t gi = (((size_t)l0 * X.n[1] + l1) * X.n[2] + l2) * 2;
                const R gr = grid[gi], gim = grid[gi + 1];
                const R w = ps[t0];
                sr = fma(w, gr, sr);
                si = fma(w, gim, si);
                if constexpr (GRAD) {
                    const R dw = dp[t0];
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
#pragma unroll
        for (int q = 0; q < 2 * NO; ++q) v[q] = det_wave_sum(v[q]);
        if (lane < 2 * NO) {
            R mine = v[0];
#pragma unroll
            for (int q = 1; q < 2 * NO; ++q) mine = lane == q ? v[q] : mine;
            outs[pos * (2 * NO) + lane] = mine;
        }
    }
}

// ---------------------------------------------------------------------------
template <typename R>
hipError_t launch_spread_det(int m, const Xform *dxf, const SItem *items, int nitems, int max_cells,
                             const unsigned char *rec, size_t rec_bytes, const R *fs, const int *cell_start,
                             hipStream_t s)
{
    if (nitems <= 0) return hipSuccess;
    const size_t lds = (size_t)max_cells * 16;
    hipError_t e = hipFuncSetAttribute((const void *)k_spread_det<R>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_spread_det<R>, dim3(nitems), dim3(64), lds, s, dxf, items, m, rec, (int)rec_bytes, fs,
                       cell_start);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_interp_det(int m, bool grad, const Xform *dxf, int B, long long Mtot, const unsigned char *rec,
                             size_t rec_bytes, R *outs, int cus, hipStream_t s)
{
    if (Mtot <= 0) return hipSuccess;
    const long long waves = std::min<long long>(Mtot, (long long)cus * 64);
    const unsigned blocks = (unsigned)((waves + 3) / 4);
    auto kern = grad ? k_interp_det<R, true> : k_interp_det<R, false>;
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(256), 0, s, dxf, B, Mtot, m, rec, (int)rec_bytes, outs);
    return hipGetLastError();
}

template hipError_t launch_spread_det<double>(int, const Xform *, const SItem *, int, int, const unsigned char *,
                                              size_t, const double *, const int *, hipStream_t);
template hipError_t launch_spread_det<float>(int, const Xform *, const SItem *, int, int, const unsigned char *,
                                             size_t, const float *, const int *, hipStream_t);
template hipError_t launch_interp_det<double>(int, bool, const Xform *, int, long long, const unsigned char *,
                                              size_t, double *, int, hipStream_t);
template hipError_t launch_interp_det<float>(int, bool, const Xform *, int, long long, const unsigned char *, size_t,
                                             float *, int, hipStream_t);

}  // namespace hpnfft
