// Device-side construction of the spread / interpolation work list.
//
// Cost of a (tile, slab) pair = points its runs sweep (each point counted
// once per segment) + one unit per run (a run is a block of lines).  Pairs heavier than a cap derived
// from the total cost are cut into runs of consecutive lines, so a clustered
// point set (many points in few tiles) still spreads evenly over the compute
// units.  The list is built without a host round trip.
#include "internal.h"

namespace hpnfft {

__device__ inline void seg_range_i(int U, int z0, int zs, int m, int n0, int *a, int *b)
{
    int lo = z0 - m - U;
    int hi = z0 + zs + m - 2 - U;
    *a = lo < 0 ? 0 : lo;
    *b = hi > n0 - 1 ? n0 - 1 : hi;
}

// Cost of one run (a block of BW lines; cs_line = its first key's start).
__device__ inline int line_cost(const int *cs_line, int n0, int z0, int zs, int m, int BW)
{
    int c = 1;
    for (int s = -1; s <= 1; ++s) {
        int a, b;
        seg_range_i(s * n0, z0, zs, m, n0, &a, &b);
        if (a <= b) c += cs_line[(b + 1) * BW] - cs_line[a * BW];
    }
    return c;
}

// One thread per (tile, slab, run): the run's cost goes to
// lcost[(tile * nslab + slab) * nl + run] (consecutive threads, consecutive
// words) and into the grand total (one atomic per workgroup: atomics on one
// address serialise).
constexpr int kCostThreads = 1024;
__global__ __launch_bounds__(kCostThreads) void k_tile_cost(const int *__restrict__ cell_start, int n0, int T,
                                                            int Zs, int m, int BW, int nslab, long long n,
                                                            int *__restrict__ lcost,
                                                            unsigned long long *__restrict__ total)
{
    __shared__ int wsum[kCostThreads / 64];
    const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int nl = T * T / BW;
    int c = 0;
    if (g < n) {
        const int li = (int)(g % nl);
        const long long ts = g / nl;
        const int slab = (int)(ts % nslab), tile = (int)(ts / nslab);
        const int z0 = slab * Zs, zs = min(Zs, n0 - z0);
        c = line_cost(cell_start + ((long long)tile * nl + li) * n0 * BW, n0, z0, zs, m, BW);
        lcost[g] = c;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += (unsigned long long)wsum[w];
        if (t) atomicAdd(total, t);
    }
}

// One wavefront per (tile, slab), kItemWaves per workgroup: the run costs
// (from k_tile_cost) are prefix-summed across the lanes and the pair is cut
// wherever the running cost crosses a multiple of the cap (a pair within the
// cap becomes one item).  The workgroup counts its items first and reserves
// their slots in the list with one atomic.
constexpr int kItemWaves = 16;
__global__ __launch_bounds__(kItemWaves * 64) void k_make_items(const int *__restrict__ lcost, int xf, int T, int BW,
                                                                int ntiles, int nslab,
                                                                const unsigned long long *__restrict__ total,
                                                                int cap_div, int min_cap, int max_items,
                                                                SItem *__restrict__ items, int *__restrict__ nitems,
                                                                int *__restrict__ overflow)
{
    __shared__ int wcount[kItemWaves], wbase[kItemWaves];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int g = blockIdx.x * kItemWaves + w;
    const bool valid = g < ntiles * nslab;
    const int tile = valid ? g / nslab : 0, slab = valid ? g % nslab : 0;
    const long long capl = (long long)(*total / (unsigned long long)cap_div);
    const int cap = capl < min_cap ? min_cap : (int)capl;
    const int nl = T * T / BW;
    const int *lc_pair = lcost + (long long)(valid ? g : 0) * nl;
    int c = 0;
    if (valid)
        for (int li = lane; li < nl; li += 64) c += lc_pair[li];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    const bool any = valid && c > nl;  // points in some run of this pair
    const bool split = any && c > cap;

    // calls f(lb, le) for every item of the pair, in order
    auto items_of = [&](auto &&f) {
        if (!any) return;
        if (!split) {
            f(0, nl);
            return;
        }
        int carry = 0;  // cost before this block of 64 runs
        int lb = 0;     // start of the open item
        for (int base = 0; base < nl; base += 64) {
            const int li = base + lane;
            const int lc = li < nl ? lc_pair[li] : 0;
            int incl = lc;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const int y = __shfl_up(incl, o, 64);
                if (lane >= o) incl += y;
            }
            const int before = carry + incl - lc, after = carry + incl;
            // a cut after run li when the running cost crosses a multiple of cap
            const bool cut = li < nl && (after / cap) != (before / cap) && li + 1 < nl;
            unsigned long long mask = __ballot(cut);
            while (mask) {
                const int k = __ffsll((long long)mask) - 1;
                mask &= mask - 1;
                f(lb, base + k + 1);
                lb = base + k + 1;
            }
            carry += __shfl(incl, 63, 64);
        }
        f(lb, nl);
    };
    int nit = 0;
    items_of([&](int, int) { ++nit; });
    if (lane == 0) wcount[w] = nit;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int k = 0; k < kItemWaves; ++k) {
            wbase[k] = t;
            t += wcount[k];
        }
        const int base = t ? atomicAdd(nitems, t) : 0;
        for (int k = 0; k < kItemWaves; ++k) wbase[k] += base;
    }
    __syncthreads();
    int idx = wbase[w];
    items_of([&](int lb, int le) {
        if (lane == 0) {
            if (idx < max_items) {
                SItem itm;
                itm.xf = xf;
                itm.tile = tile;
                itm.slab = slab;
                itm.lb = lb;
                itm.le = le;
                itm.pad0 = itm.pad1 = itm.pad2 = 0;
                items[idx] = itm;
            } else {
                atomicOr(overflow, 1);
            }
        }
        ++idx;
    });
}

hipError_t launch_tile_cost(const int *cell_start, const Xform &X, int T, int Zs, int m, int *lcost,
                            unsigned long long *total, hipStream_t s)
{
    const int BW = block_w(2 * m);
    const long long n = (long long)X.ntx * X.nty * X.nslab * (T * T / BW);
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tile_cost, dim3((unsigned)((n + kCostThreads - 1) / kCostThreads)), dim3(kCostThreads), 0, s,
                       cell_start, X.n[0], T, Zs, m, BW, X.nslab, n, lcost, total);
    return hipGetLastError();
}

hipError_t launch_make_items(const int *lcost, int xf, const Xform &X, int T, int m, const unsigned long long *total,
                             int cap_div, int min_cap, int max_items, SItem *items, int *nitems, int *overflow,
                             hipStream_t s)
{
    const long long pairs = (long long)X.ntx * X.nty * X.nslab;  // one wavefront per pair
    if (pairs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_make_items, dim3((unsigned)((pairs + kItemWaves - 1) / kItemWaves)), dim3(kItemWaves * 64), 0, s,
                       lcost, xf, T,
                       block_w(2 * m), X.ntx * X.nty, X.nslab, total, cap_div, min_cap, max_items, items, nitems,
                       overflow);
    return hipGetLastError();
}

}  // namespace hpnfft
