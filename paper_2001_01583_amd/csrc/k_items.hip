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

// One workgroup per (tile, slab): its threads sum the line costs, the total
// is stored in tcost (no zeroing needed) and added to the grand total.
__global__ __launch_bounds__(256) void k_tile_cost(const int *__restrict__ cell_start, int n0, int T, int Zs,
                                                   int m, int BW, int nslab, int *__restrict__ tcost,
                                                   unsigned long long *__restrict__ total)
{
    __shared__ int blk;
    if (threadIdx.x == 0) blk = 0;
    __syncthreads();
    const int ts = blockIdx.x;
    const int slab = ts % nslab, tile = ts / nslab;
    const int z0 = slab * Zs, zs = min(Zs, n0 - z0);
    const int nl = T * T / BW;
    int c = 0;
    for (int li = threadIdx.x; li < nl; li += blockDim.x)
        c += line_cost(cell_start + ((long long)tile * nl + li) * n0 * BW, n0, z0, zs, m, BW);
    // wavefront sum, then one LDS add per wavefront
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0) atomicAdd(&blk, c);
    __syncthreads();
    if (threadIdx.x == 0) {
        tcost[ts] = blk;
        atomicAdd(total, (unsigned long long)blk);
    }
}

// One wavefront per (tile, slab): the T*T line costs are prefix-summed across
// the lanes and the pair is cut wherever the running cost crosses a multiple of
// the cap (a pair within the cap becomes one item).
__global__ void k_make_items(const int *__restrict__ cell_start, int xf, int n0, int T, int Zs, int m, int BW,
                             int ntiles, int nslab, const int *__restrict__ tcost,
                             const unsigned long long *__restrict__ total, int cap_div, int min_cap,
                             int max_items, SItem *__restrict__ items, int *__restrict__ nitems,
                             int *__restrict__ overflow)
{
    const int lane = threadIdx.x & 63;
    const int g = (int)(((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    if (g >= ntiles * nslab) return;
    const int tile = g / nslab, slab = g % nslab;
    const int z0 = slab * Zs, zs = min(Zs, n0 - z0);
    long long capl = (long long)(*total / (unsigned long long)cap_div);
    const int cap = capl < min_cap ? min_cap : (int)capl;
    const int c = tcost[g];
    const int nl = T * T / BW;
    auto emit = [&](int lb, int le) {
        int idx = atomicAdd(nitems, 1);
        if (idx >= max_items) {
            atomicOr(overflow, 1);
            return;
        }
        SItem itm;
        itm.xf = xf;
        itm.tile = tile;
        itm.slab = slab;
        itm.lb = lb;
        itm.le = le;
        itm.pad0 = itm.pad1 = itm.pad2 = 0;
        items[idx] = itm;
    };
    if (c <= nl) return;  // no points in any line of this pair
    if (c <= cap) {
        if (lane == 0) emit(0, nl);
        return;
    }
    // lines in consecutive blocks of 64: lane k of block handles line base + k
    int carry = 0;       // cost before this block
    int lb = 0;          // start of the open item
    for (int base = 0; base < nl; base += 64) {
        int li = base + lane;
        int lc = li < nl ? line_cost(cell_start + ((long long)tile * nl + li) * n0 * BW, n0, z0, zs, m, BW) : 0;
        int incl = lc;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            int y = __shfl_up(incl, o, 64);
            if (lane >= o) incl += y;
        }
        int before = carry + incl - lc, after = carry + incl;
        // a cut after line li when the running cost crosses a multiple of cap
        bool cut = li < nl && (after / cap) != (before / cap) && li + 1 < nl;
        unsigned long long mask = __ballot(cut);
        while (mask) {
            int k = __ffsll((long long)mask) - 1;
            mask &= mask - 1;
            int le = base + k + 1;
            if (lane == 0) emit(lb, le);
            lb = le;
        }
        carry += __shfl(incl, 63, 64);
    }
    if (lane == 0 && lb < nl) emit(lb, nl);
}

hipError_t launch_tile_cost(const int *cell_start, const Xform &X, int T, int Zs, int m, int *tcost,
                            unsigned long long *total, hipStream_t s)
{
    const long long nts = (long long)X.ntx * X.nty * X.nslab;
    if (nts <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tile_cost, dim3((unsigned)nts), dim3(256), 0, s, cell_start, X.n[0], T, Zs, m,
                       block_w(2 * m), X.nslab, tcost, total);
    return hipGetLastError();
}

hipError_t launch_make_items(const int *cell_start, int xf, const Xform &X, int T, int Zs, int m,
                             const int *tcost, const unsigned long long *total, int cap_div, int min_cap,
                             int max_items, SItem *items, int *nitems, int *overflow, hipStream_t s)
{
    long long n = (long long)X.ntx * X.nty * X.nslab * 64;  // one wavefront per pair
    hipLaunchKernelGGL(k_make_items, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, cell_start, xf, X.n[0],
                       T, Zs, m, block_w(2 * m), X.ntx * X.nty, X.nslab, tcost, total, cap_div, min_cap,
                       max_items, items, nitems, overflow);
    return hipGetLastError();
}

}  // namespace hpnfft
