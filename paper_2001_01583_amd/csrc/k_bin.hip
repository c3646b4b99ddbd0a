// Point binning ("set_points"): cell index and offset of every point, a
// counting sort of the points by cell, and tabulation of the window values.
//
// The paper's spreading kernel assigns one thread per point and resolves
// collisions with atomic additions (Section 3, Spreading step).  Here the
// points are first sorted so that every z-line of grid cells (fixed cells in
// dims 1 and 2) holds a contiguous, plane-ordered run of points; the spread
// and interpolation kernels then sweep those runs with register windows.
//
// Sort key of a point with cell (c0, c1, c2):
//   tile  = (c1 / T) * ntx + (c2 / T)
//   line  = tile * T*T + (c1 % T) * T + (c2 % T)
//   key   = line * n0 + c0
#include "internal.h"
#include "window.h"

namespace hpnfft {

__device__ inline int wrap_cell(int c, int n)
{
    c %= n;
    return c < 0 ? c + n : c;
}

// Cell (storage index in [0, n)) and offset u in [0, 1) of one coordinate;
// sets *bad for a coordinate outside [-1/2, 1/2) or not finite.
__device__ inline int cell_of(double xv, int n, double *u, bool *bad)
{
    if (!(xv >= -0.5 && xv < 0.5)) {  // NaN fails both comparisons
        *bad = true;
        xv = 0.0;
    }
    double v = xv * (double)n;
    double fl = floor(v);
    *u = v - fl;                       // exact
    return wrap_cell((int)fl, n);
}

__device__ inline int sort_key(const int c[3], int T, int ntx, int n0)
{
    int tile = (c[1] / T) * ntx + (c[2] / T);
    int line = tile * T * T + (c[1] % T) * T + (c[2] % T);
    return line * n0 + c[0];
}

template <typename XT>
__global__ void k_bin_count(const XT *__restrict__ x, long long M, int n0, int n1, int n2,
                            int T, int ntx, int *__restrict__ counts, int *__restrict__ rank,
                            int *__restrict__ err)
{
    long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    const int n[3] = {n0, n1, n2};
    bool bad = false;
    int c[3];
    for (int t = 0; t < 3; ++t) {
        double u;
        c[t] = cell_of((double)x[j * 3 + t], n[t], &u, &bad);
    }
    if (bad) atomicOr(err, 1);
    rank[j] = atomicAdd(&counts[sort_key(c, T, ntx, n0)], 1);
}

template <typename XT>
__global__ void k_bin_scatter(const XT *__restrict__ x, long long M, long long poff, int n0, int n1,
                              int n2, int T, int ntx, const int *__restrict__ cell_start,
                              const int *__restrict__ rank, int *__restrict__ perm,
                              unsigned char *__restrict__ rec, size_t rec_bytes, size_t off_pz,
                              double *__restrict__ us)
{
    long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    const int n[3] = {n0, n1, n2};
    bool bad = false;
    int c[3];
    double u[3];
    for (int t = 0; t < 3; ++t) c[t] = cell_of((double)x[j * 3 + t], n[t], &u[t], &bad);
    long long pos = poff + cell_start[sort_key(c, T, ntx, n0)] + rank[j];
    perm[pos] = (int)(poff + j);
    *reinterpret_cast<int *>(rec + pos * rec_bytes + off_pz) = c[0];
    us[pos * 3 + 0] = u[0];
    us[pos * 3 + 1] = u[1];
    us[pos * 3 + 2] = u[2];
}

// Window values of the sorted points, one thread per (point, dimension, tap),
// written into the point records (consecutive threads write consecutive
// words).  Tap t (0..2m-1) of a point in cell c with offset u sits on grid
// cell c - m + 1 + t, at grid-unit distance u + m - 1 - t.  Along dim 0 the
// taps are stored rotated: slot s = (c0 - m + 1 + t) mod 2m, so that a
// register window indexed by plane mod 2m needs no per-point shuffling.
template <typename R>
__global__ void k_psi(const double *__restrict__ us, long long M, long long poff, int m, double b,
                      double inv_peak, int n0, int n1, int n2, unsigned char *__restrict__ rec,
                      size_t rec_bytes, int grad)
{
    const int M2 = 2 * m;
    long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= M * 3 * M2) return;
    long long p = poff + g / (3 * M2);
    int rem = (int)(g % (3 * M2));
    int dim = rem / M2, t = rem - dim * M2;
    unsigned char *rp = rec + p * rec_bytes;
    double u = us[p * 3 + dim];
    int s = t;
    if (dim == 0) {
        int c0 = *reinterpret_cast<const int *>(rp + rec_off_pz(M2, sizeof(R)));
        int r = (c0 - m + 1) % M2;
        s = t + (r < 0 ? r + M2 : r);
        if (s >= M2) s -= M2;
    }
    double nd = dim == 0 ? n0 : (dim == 1 ? n1 : n2);
    double dist = u + (double)(m - 1 - t);
    // evaluated in float64 for both paths (the float path stores the values
    // rounded once)
    R *dst = reinterpret_cast<R *>(rp) + dim * M2 + s;
    *dst = (R)kb_phi(dist, m, b, inv_peak);
    if (grad)
        *(reinterpret_cast<R *>(rp + rec_prefix(M2, sizeof(R))) + dim * M2 + s) =
            (R)(nd * kb_dphi(dist, m, b, inv_peak));
}

// ---------------------------------------------------------------------------
// Exclusive prefix sum (in place) over int counts: per-block reduce, scan of
// the block sums (recursively), then a per-block scan with the block offset.
constexpr int kScanThreads = 256;
constexpr int kScanPer = 16;
constexpr int kScanBlock = kScanThreads * kScanPer;  // 4096 elements

__device__ inline int block_exclusive_scan(int v, int *sh, int *total)
{
    // Hillis-Steele over the block's 256 thread sums in LDS.
    int tid = threadIdx.x;
    sh[tid] = v;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        int add = tid >= off ? sh[tid - off] : 0;
        __syncthreads();
        sh[tid] += add;
        __syncthreads();
    }
    int incl = sh[tid];
    *total = sh[kScanThreads - 1];
    __syncthreads();
    return incl - v;
}

__global__ void k_scan_reduce(const int *__restrict__ data, long long n, int *__restrict__ sums)
{
    __shared__ int sh[kScanThreads];
    long long base = (long long)blockIdx.x * kScanBlock + (long long)threadIdx.x * kScanPer;
    int s = 0;
    for (int i = 0; i < kScanPer; ++i)
        if (base + i < n) s += data[base + i];
    int total;
    block_exclusive_scan(s, sh, &total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ void k_scan_apply(int *__restrict__ data, long long n, const int *__restrict__ offs)
{
    __shared__ int sh[kScanThreads];
    long long base = (long long)blockIdx.x * kScanBlock + (long long)threadIdx.x * kScanPer;
    int v[kScanPer];
    int s = 0;
    for (int i = 0; i < kScanPer; ++i) {
        v[i] = base + i < n ? data[base + i] : 0;
        s += v[i];
    }
    int total;
    int run = block_exclusive_scan(s, sh, &total) + (offs ? offs[blockIdx.x] : 0);
    for (int i = 0; i < kScanPer; ++i) {
        if (base + i < n) data[base + i] = run;
        run += v[i];
    }
}

hipError_t launch_scan(int *data, long long n, int *tmp, hipStream_t s)
{
    long long nb = (n + kScanBlock - 1) / kScanBlock;
    if (nb <= 1) {
        hipLaunchKernelGGL(k_scan_apply, dim3(1), dim3(kScanThreads), 0, s, data, n, (const int *)nullptr);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanThreads), 0, s, data, n, tmp);
    hipError_t e = launch_scan(tmp, nb, tmp + nb, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kScanThreads), 0, s, data, n, tmp);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
hipError_t launch_bin_count(const double *x, const float *xf32, long long M, const Xform &X, int T,
                            int m, int *counts, int *rank, int *err, hipStream_t s)
{
    (void)m;
    unsigned nb = (unsigned)((M + 255) / 256);
    if (x)
        hipLaunchKernelGGL(k_bin_count<double>, dim3(nb), dim3(256), 0, s, x, M, X.n[0], X.n[1],
                           X.n[2], T, X.ntx, counts, rank, err);
    else
        hipLaunchKernelGGL(k_bin_count<float>, dim3(nb), dim3(256), 0, s, xf32, M, X.n[0], X.n[1],
                           X.n[2], T, X.ntx, counts, rank, err);
    return hipGetLastError();
}

hipError_t launch_bin_scatter(const double *x, const float *xf32, long long M, const Xform &X, int T,
                              int m, const int *cell_start, const int *rank, int *perm, unsigned char *rec,
                              size_t rec_bytes, size_t off_pz, double *us, hipStream_t s)
{
    (void)m;
    unsigned nb = (unsigned)((M + 255) / 256);
    if (x)
        hipLaunchKernelGGL(k_bin_scatter<double>, dim3(nb), dim3(256), 0, s, x, M, X.poff, X.n[0],
                           X.n[1], X.n[2], T, X.ntx, cell_start, rank, perm, rec, rec_bytes, off_pz, us);
    else
        hipLaunchKernelGGL(k_bin_scatter<float>, dim3(nb), dim3(256), 0, s, xf32, M, X.poff, X.n[0],
                           X.n[1], X.n[2], T, X.ntx, cell_start, rank, perm, rec, rec_bytes, off_pz, us);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_psi(const double *us, long long M, long long poff, const Xform &X, int m, double b,
                      double inv_peak, unsigned char *rec, size_t rec_bytes, bool grad, hipStream_t s)
{
    unsigned nb = (unsigned)((M * 3 * 2 * m + 255) / 256);
    hipLaunchKernelGGL(k_psi<R>, dim3(nb), dim3(256), 0, s, us, M, poff, m, b, inv_peak, X.n[0], X.n[1],
                       X.n[2], rec, rec_bytes, grad ? 1 : 0);
    return hipGetLastError();
}

template hipError_t launch_psi<double>(const double *, long long, long long, const Xform &, int, double,
                                       double, unsigned char *, size_t, bool, hipStream_t);
template hipError_t launch_psi<float>(const double *, long long, long long, const Xform &, int, double,
                                      double, unsigned char *, size_t, bool, hipStream_t);

}  // namespace hpnfft
