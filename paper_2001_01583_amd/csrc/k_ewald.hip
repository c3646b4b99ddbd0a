// Real-space Ewald sum of Eq. (11) (Section 5) with cell lists, for the
// large ionic systems of the paper's HP-ENUF timing experiment (up to
// 12 * 64^3 ions).  The reciprocal part (Eq. (12)) runs through the NFFT.
//
// The box of side L is cut into nc^3 cubic cells of side h = L / nc >= rcut,
// so every pair closer than rcut lies in the same or a neighbouring cell.
// Ions are counting-sorted by cell (count, scan, scatter, then input order
// within each cell) into one float64 (x, y, z, q) record each.  One workgroup per cell: each thread holds one
// ion of the cell, the 27 neighbour cells stream through LDS in tiles, and
// a neighbour across the periodic boundary is shifted by L on the way in, so
// every pair is seen once per ion with its nearest image.  Each ion's force
// has a single writer; the energy is reduced per cell in float64 and summed
// in a fixed order.
#include "internal.h"

namespace hpnfft {

constexpr int kPairThreads = 128;
constexpr int kPairTile = 256;

// Wrap into [0, L) and return the cell coordinate along one axis.
__device__ inline double wrap_box(double v, double L)
{
    v -= L * floor(v / L);
    return v >= L ? v - L : v;  // rounding can leave exactly L
}
__device__ inline int cell_axis(double v, double inv_h, int nc)
{
    const int c = (int)(v * inv_h);
    return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

__global__ __launch_bounds__(256) void k_cells_count(const double *__restrict__ r, long long M, double L, int nc,
                                                     int *__restrict__ counts, int *__restrict__ cell,
                                                     int *__restrict__ rank)
{
    const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    const double inv_h = nc / L;
    const int cx = cell_axis(wrap_box(r[3 * j], L), inv_h, nc);
    const int cy = cell_axis(wrap_box(r[3 * j + 1], L), inv_h, nc);
    const int cz = cell_axis(wrap_box(r[3 * j + 2], L), inv_h, nc);
    const int c = (cx * nc + cy) * nc + cz;
    cell[j] = c;
    rank[j] = atomicAdd(&counts[c], 1);
}

__global__ __launch_bounds__(256) void k_cells_scatter(const double *__restrict__ r, const double *__restrict__ q,
                                                       long long M, double L, const int *__restrict__ start,
                                                       const int *__restrict__ cell, const int *__restrict__ rank,
                                                       double4 *__restrict__ sorted, int *__restrict__ orig)
{
    const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    const int pos = start[cell[j]] + rank[j];
    sorted[pos] = make_double4(wrap_box(r[3 * j], L), wrap_box(r[3 * j + 1], L), wrap_box(r[3 * j + 2], L), q[j]);
    orig[pos] = (int)j;
}

// The scatter's order within a cell follows its atomic ranks, which vary from
// run to run.  This pass puts each cell's ions in the order of their input
// index (rank = ions of the cell with a smaller index), so the pair sums, and
// the results bit for bit, do not depend on that order.  Work per cell is the
// square of its ion count (about 150 at the sweep's densities).
__global__ __launch_bounds__(256) void k_cells_reorder(const double4 *__restrict__ sorted_tmp,
                                                       const int *__restrict__ orig_tmp,
                                                       const int *__restrict__ start,
                                                       double4 *__restrict__ sorted, int *__restrict__ orig)
{
    const int c = blockIdx.x;
    const int s0 = start[c], s1 = start[c + 1];
    for (int i = s0 + threadIdx.x; i < s1; i += blockDim.x) {
        const int oi = orig_tmp[i];
        int r = 0;
        for (int j = s0; j < s1; ++j) r += orig_tmp[j] < oi;
        sorted[s0 + r] = sorted_tmp[i];
        orig[s0 + r] = oi;
    }
}

// U = 1/2 sum_i sum_{j != i, r_ij < rcut} q_i q_j erfc(alpha r_ij) / r_ij and
// F_i = sum_j q_i q_j [erfc(alpha r)/r + 2 alpha/sqrt(pi) exp(-alpha^2 r^2)] d_ij / r^2.
__global__ __launch_bounds__(kPairThreads) void k_cells_pairs(const double4 *__restrict__ sorted,
                                                              const int *__restrict__ orig,
                                                              const int *__restrict__ start, int nc, double L,
                                                              double alpha, double rcut2,
                                                              double *__restrict__ part,
                                                              double *__restrict__ forces)
{
    __shared__ double4 tile[kPairTile];
    __shared__ double red[kPairThreads];
    const int c = blockIdx.x;
    const int cz = c % nc, cy = (c / nc) % nc, cx = c / (nc * nc);
    const int s0 = start[c], s1 = start[c + 1];
    const double c2 = 2.0 * alpha / sqrt(M_PI);
    double e_acc = 0.0;
    for (int ib = s0; ib < s1; ib += kPairThreads) {
        const int i = ib + threadIdx.x;
        const bool vi = i < s1;
        const double4 pi = vi ? sorted[i] : make_double4(0.0, 0.0, 0.0, 0.0);
        double fx = 0.0, fy = 0.0, fz = 0.0, e = 0.0;
        for (int nb = 0; nb < 27; ++nb) {
            int ax = cx + nb / 9 - 1, ay = cy + (nb / 3) % 3 - 1, az = cz + nb % 3 - 1;
            double sx = 0.0, sy = 0.0, sz = 0.0;
            if (ax < 0) { ax += nc; sx = -L; } else if (ax >= nc) { ax -= nc; sx = L; }
            if (ay < 0) { ay += nc; sy = -L; } else if (ay >= nc) { ay -= nc; sy = L; }
            if (az < 0) { az += nc; sz = -L; } else if (az >= nc) { az -= nc; sz = L; }
            const int a = (ax * nc + ay) * nc + az;
            const int t0 = start[a], t1 = start[a + 1];
            for (int tb = t0; tb < t1; tb += kPairTile) {
                const int cnt = min(kPairTile, t1 - tb);
                __syncthreads();
                for (int k = threadIdx.x; k < cnt; k += kPairThreads) {
                    double4 v = sorted[tb + k];
                    v.x += sx;
                    v.y += sy;
                    v.z += sz;
                    tile[k] = v;
                }
                __syncthreads();
                if (!vi) continue;
                for (int k = 0; k < cnt; ++k) {
                    if (nb == 13 && tb + k == i) continue;  // the ion itself (own cell, no shift)
                    const double4 pj = tile[k];
                    const double dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
                    const double d2 = dx * dx + dy * dy + dz * dz;
                    if (d2 >= rcut2) continue;
                    const double d = sqrt(d2);
                    const double qq = pi.w * pj.w;
                    const double ec = erfc(alpha * d) / d;
                    e += 0.5 * qq * ec;
                    const double g = qq * (ec + c2 * exp(-alpha * alpha * d2)) / d2;
                    fx += g * dx;
                    fy += g * dy;
                    fz += g * dz;
                }
            }
        }
        if (vi && forces) {
            const long long o = orig[i];
            forces[3 * o] = fx;
            forces[3 * o + 1] = fy;
            forces[3 * o + 2] = fz;
        }
        e_acc += e;
    }
    red[threadIdx.x] = e_acc;
    __syncthreads();
    for (int off = kPairThreads / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[c] = red[0];
}

// Workspace of the cell-list sum: [starts: nc^3 + 1 ints][scan scratch]
// [cell, rank, orig, orig in scatter order: M ints each][sorted ions, and in
// scatter order: M x 32 B each][cell partials: nc^3 doubles], each region
// 256-byte aligned.
static size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }
static size_t scan_tmp_ints(long long n)
{
    const long long nb = (n + 4095) / 4096;
    return (size_t)(nb + nb / 2048 + 64);
}
CellsLayout cells_layout(long long M, int nc)
{
    CellsLayout C{};
    const long long ncell = (long long)nc * nc * nc;
    size_t off = 0;
    C.start = off;
    off = al256(off + (size_t)(ncell + 1) * 4);
    C.scan = off;
    off = al256(off + scan_tmp_ints(ncell + 1) * 4);
    C.cell = off;
    off = al256(off + (size_t)M * 4);
    C.rank = off;
    off = al256(off + (size_t)M * 4);
    C.orig = off;
    off = al256(off + (size_t)M * 4);
    C.orig_tmp = off;
    off = al256(off + (size_t)M * 4);
    C.sorted = off;
    off = al256(off + (size_t)M * 32);
    C.sorted_tmp = off;
    off = al256(off + (size_t)M * 32);
    C.part = off;
    off = al256(off + (size_t)ncell * 8);
    C.total = off;
    return C;
}

hipError_t launch_ewald_cells(const double *r, const double *q, long long M, double L, double alpha, double rcut,
                              int nc, unsigned char *ws, double *energy, double *forces, hipStream_t s)
{
    const CellsLayout C = cells_layout(M, nc);
    const long long ncell = (long long)nc * nc * nc;
    int *start = reinterpret_cast<int *>(ws + C.start);
    hipError_t e = launch_zero(start, (size_t)(ncell + 1) * 4, s);
    if (e != hipSuccess) return e;
    const unsigned nb = (unsigned)((M + 255) / 256);
    int *cell = reinterpret_cast<int *>(ws + C.cell), *rank = reinterpret_cast<int *>(ws + C.rank);
    int *orig = reinterpret_cast<int *>(ws + C.orig), *orig_tmp = reinterpret_cast<int *>(ws + C.orig_tmp);
    double4 *sorted = reinterpret_cast<double4 *>(ws + C.sorted);
    double4 *sorted_tmp = reinterpret_cast<double4 *>(ws + C.sorted_tmp);
    double *part = reinterpret_cast<double *>(ws + C.part);
    hipLaunchKernelGGL(k_cells_count, dim3(nb), dim3(256), 0, s, r, M, L, nc, start, cell, rank);
    e = launch_scan(start, ncell + 1, reinterpret_cast<int *>(ws + C.scan), s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cells_scatter, dim3(nb), dim3(256), 0, s, r, q, M, L, start, cell, rank, sorted_tmp,
                       orig_tmp);
    hipLaunchKernelGGL(k_cells_reorder, dim3((unsigned)ncell), dim3(256), 0, s, sorted_tmp, orig_tmp, start, sorted,
                       orig);
    hipLaunchKernelGGL(k_cells_pairs, dim3((unsigned)ncell), dim3(kPairThreads), 0, s, sorted, orig, start, nc, L,
                       alpha, rcut * rcut, part, forces);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_sum_partials(part, (int)ncell, energy, s);
}

}  // namespace hpnfft
