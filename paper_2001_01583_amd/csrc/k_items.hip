// Device-side construction of the spread / interpolation work list.
//
// Cost of a (tile, slab) pair = points its lines sweep (each point counted
// once per segment) + one unit per line.  Pairs heavier than a cap derived
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

__device__ inline int line_cost(const int *cs_line, int n0, int z0, int zs, int m)
{
    int c = 1;
    for (int s = -1; s <= 1; ++s) {
        int a, b;
        seg_range_i(s * n0, z0, zs, m, n0, &a, &b);
        if (a <= b) c += cs_line[b + 1] - cs_line[a];
    }
    return c;
}

__global__ void k_tile_cost(const int *__restrict__ cell_start, int n0, int T, int Zs, int m,
                            int ntiles, int nslab, int *__restrict__ tcost,
                            unsigned long long *__restrict__ total)
{
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ntiles * nslab) return;
    int tile = g / nslab, slab = g % nslab;
    int z0 = slab * Zs, zs = min(Zs, n0 - z0);
    int c = 0;
    for (int li = 0; li < T * T; ++li)
        c += line_cost(cell_start + ((long long)tile * T * T + li) * n0, n0, z0, zs, m);
    tcost[g] = c;
    atomicAdd(total, (unsigned long long)c);
}

__global__ void k_make_items(const int *__restrict__ cell_start, int xf, int n0, int T, int Zs, int m,
                             int ntiles, int nslab, const int *__restrict__ tcost,
                             const unsigned long long *__restrict__ total, int cap_div, int min_cap,
                             int max_items, SItem *__restrict__ items, int *__restrict__ nitems,
                             int *__restrict__ overflow)
{
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ntiles * nslab) return;
    int tile = g / nslab, slab = g % nslab;
    int z0 = slab * Zs, zs = min(Zs, n0 - z0);
    long long capl = (long long)(*total / (unsigned long long)cap_div);
    int cap = capl < min_cap ? min_cap : (int)capl;
    int c = tcost[g];
    // a pair whose lines hold no points is skipped entirely
    if (c <= T * T) return;
    auto emit = [&](int lb, int le) {
        int idx = atomicAdd(nitems, 1);
        if (idx >= max_items) {
            atomicOr(overflow, 1);
            return;
        }
        SItem it;
        it.xf = xf;
        it.tile = tile;
        it.slab = slab;
        it.lb = lb;
        it.le = le;
        it.pad0 = it.pad1 = it.pad2 = 0;
        items[idx] = it;
    };
    if (c <= cap) {
        emit(0, T * T);
        return;
    }
    int lb = 0, acc = 0;
    for (int li = 0; li < T * T; ++li) {
        acc += line_cost(cell_start + ((long long)tile * T * T + li) * n0, n0, z0, zs, m);
        if (acc >= cap) {
            emit(lb, li + 1);
            lb = li + 1;
            acc = 0;
        }
    }
    if (lb < T * T && acc > 0) emit(lb, T * T);
}

hipError_t launch_tile_cost(const int *cell_start, const Xform &X, int T, int Zs, int m, int *tcost,
                            unsigned long long *total, hipStream_t s)
{
    int n = X.ntx * X.nty * X.nslab;
    hipLaunchKernelGGL(k_tile_cost, dim3((n + 127) / 128), dim3(128), 0, s, cell_start, X.n[0], T, Zs, m,
                       X.ntx * X.nty, X.nslab, tcost, total);
    return hipGetLastError();
}

hipError_t launch_make_items(const int *cell_start, int xf, const Xform &X, int T, int Zs, int m,
                             const int *tcost, const unsigned long long *total, int cap_div, int min_cap,
                             int max_items, SItem *items, int *nitems, int *overflow, hipStream_t s)
{
    int n = X.ntx * X.nty * X.nslab;
    hipLaunchKernelGGL(k_make_items, dim3((n + 127) / 128), dim3(128), 0, s, cell_start, xf, X.n[0], T, Zs,
                       m, X.ntx * X.nty, X.nslab, tcost, total, cap_div, min_cap, max_items, items,
                       nitems, overflow);
    return hipGetLastError();
}

}  // namespace hpnfft
