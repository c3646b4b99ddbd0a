// Point binning ("set_points"): cell index and offset of every point, a
// counting sort of the points by cell, and tabulation of the window values.
//
// The paper's spreading kernel assigns one thread per point and resolves
// collisions with atomic additions (Section 3, Spreading step).  Here the
// points are first sorted so that every z-line of grid cells (fixed cells in
// dims 1 and 2) holds a contiguous, plane-ordered run of points; the spread
// and interpolation kernels then sweep those runs with register windows.
//
// Sort key of a point with cell (c0, c1, c2), lines grouped in blocks of BW
// lines along dim 2 (BW divides T):
//   tile  = (c1 / T) * ntx + (c2 / T)
//   block = tile * T*T/BW + (c1 % T) * T/BW + (c2 % T) / BW
//   key   = (block * n0 + c0) * BW + (c2 % T) % BW
// so a block's points are ordered by plane, then by line.  With BW = 1 a
// block is one line.
#include "internal.h"
#include "window.h"

namespace hpnfft {

// floor(x n) for x in [-1/2, 1/2) lies in [-n/2, n/2]: one conditional add
// brings it to its storage index in [0, n)
__device__ inline int wrap_cell(int c, int n) { return c < 0 ? c + n : c; }

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

// c / T and c % T for the tile edge T: a shift and a mask when T is a power
// of two (T is the same for every thread, so the branch is uniform)
__device__ inline void tile_split(int c, int T, int *q, int *r)
{
    if ((T & (T - 1)) == 0) {
        const int sh = __ffs(T) - 1;
        *q = c >> sh;
        *r = c & (T - 1);
    } else {
        *q = c / T;
        *r = c - *q * T;
    }
}

// BW is 1 or 8 (block_w) and divides T
__device__ inline int sort_key(const int c[3], int T, int ntx, int n0, int BW)
{
    int q1, r1, q2, r2;
    tile_split(c[1], T, &q1, &r1);
    tile_split(c[2], T, &q2, &r2);
    const int bsh = BW == 8 ? 3 : 0;
    const int tile = q1 * ntx + q2;
    const int block = tile * ((T * T) >> bsh) + r1 * (T >> bsh) + (r2 >> bsh);
    return (block * n0 + c[0]) * BW + (r2 & (BW - 1));
}

// Count pass: cell and sort key of every point, its rank among the points of
// its cell (the counting sort's first half), the domain check, and the
// float64 copy of the coordinates that later passes (and the tiling
// autotuner) read.  xs_out may be null when x already is that copy.
// Plans of d < 3 dimensions (flat = 3 - d leading dims without a
// coordinate) read d values per point and store three, the flat ones zero.
template <typename XT>
__global__ void k_bin_count(const XT *__restrict__ x, long long M, int n0, int n1, int n2, int T, int ntx,
                            int BW, int flat, int nb0, int nb1, int nb2, int *__restrict__ counts,
                            int *__restrict__ rank, int *__restrict__ err, double *__restrict__ xs_out,
                            int *__restrict__ keys_out)
{
    long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    const int n[3] = {n0, n1, n2};
    const int nbox[3] = {nb0, nb1, nb2};
    const int d = 3 - flat;
    bool bad = false;
    int c[3];
    double xv[3];
    for (int t = 0; t < 3; ++t) {
        xv[t] = t < flat ? 0.0 : (double)x[j * d + (t - flat)];
        double u;
        c[t] = cell_of(xv[t], n[t], &u, &bad);
    }
    if (xs_out) {
        if (flat == 0) {
            // the copy runs over the flat array (words j, j + M, j + 2M), so
            // every store instruction writes one contiguous span
#pragma unroll
            for (int t = 0; t < 3; ++t) xs_out[j + t * M] = (double)x[j + t * M];
        } else {
#pragma unroll
            for (int t = 0; t < 3; ++t) xs_out[j * 3 + t] = xv[t];
        }
    }
    if (bad) atomicOr(err, 1);
    const int key = nb0 ? box_key(c, n, nbox) : sort_key(c, T, ntx, n0, BW);
    rank[j] = atomicAdd(&counts[key], 1);
    if (keys_out) keys_out[j] = key;
}

// Scatter of the points into sorted order, with the window values of each
// point tabulated into its record on the way (one thread per point).  Tap t
// (0..2m-1) of a point in cell c with offset u sits on grid cell c - m + 1 + t,
// at grid-unit distance u + m - 1 - t.  Along dim 0 the taps are stored
// rotated: slot s holds tap (s - (c0 - m + 1)) mod 2m, so that a register
// window indexed by plane mod 2m needs no per-point shuffling.  Values are
// evaluated in float64 and rounded once for the float32 path.
typedef unsigned int v4u_bin __attribute__((ext_vector_type(4)));
typedef unsigned int v2u_bin __attribute__((ext_vector_type(2)));

// Store NB bytes from registers to a 16-byte aligned address with 16-byte
// stores (and one 8-byte store for a remainder).
template <int NB, typename T>
__device__ inline void store_block(unsigned char *dst, const T *src)
{
    const unsigned char *b = reinterpret_cast<const unsigned char *>(src);
#pragma unroll
    for (int i = 0; i < NB / 16; ++i) {
        v4u_bin v;
        __builtin_memcpy(&v, b + 16 * i, 16);
        reinterpret_cast<v4u_bin *>(dst)[i] = v;
    }
    if constexpr (NB % 16 != 0) {
        v2u_bin v;
        __builtin_memcpy(&v, b + 16 * (NB / 16), 8);
        *reinterpret_cast<v2u_bin *>(dst + 16 * (NB / 16)) = v;
    }
}

// Polynomial in v with NC coefficients (c[k] multiplies v^k), by Horner's rule.
template <int NC>
__device__ inline double horner(const double *__restrict__ c, double v)
{
    double r = c[NC - 1];
#pragma unroll
    for (int k = NC - 2; k >= 0; --k) r = fma(r, v, c[k]);
    return r;
}

// Point j's sorted position (written to perm and ipos unless the positions
// are fixed), window tables in record slot order and record header.
template <typename R, int M2, bool GRAD>
__device__ inline long long scatter_point(long long j, const double *__restrict__ xd, const float *__restrict__ xf,
                                          long long poff, int n0, int n1, int n2, int T, int ntx,
                                          const int *__restrict__ cell_start, const int *__restrict__ rank,
                                          int *__restrict__ perm, int *__restrict__ ipos, const WindowParams &wp,
                                          const double *__restrict__ poly, int flat, int nb0, int nb1, int nb2,
                                          const int *__restrict__ fixed_pos, R (&w)[3 * M2],
                                          R (&dw)[GRAD ? 3 * M2 : 1], int2 &head)
{
    constexpr int m = M2 / 2;
    constexpr int NC = sizeof(R) == 4 ? kPolyF32 : kPolyF64;
    const int n[3] = {n0, n1, n2};
    bool bad = false;
    int c[3];
    double u[3];
    for (int t = 0; t < 3; ++t) {
        const double xv = xd ? xd[j * 3 + t] : (double)xf[j * 3 + t];
        c[t] = cell_of(xv, n[t], &u[t], &bad);
    }
    const int nbox[3] = {nb0, nb1, nb2};
    const int key = nb0 ? box_key(c, n, nbox) : sort_key(c, T, ntx, n0, block_w(M2));
    long long pos;
    if (fixed_pos) {
        pos = fixed_pos[poff + j];
    } else {
        pos = poff + cell_start[key] + rank[j];
        perm[pos] = (int)(poff + j);
        ipos[poff + j] = (int)pos;
    }

    int rot = (c[0] - m + 1) % M2;
    if (rot < 0) rot += M2;
    // values in tap order (the tap index, hence the polynomial, is the same
    // for every thread).  A flat dim (no coordinate, N_t = 1) holds the unit
    // impulse on cell 0, which the point (at 0) reaches with tap m - 1.
    // Derivative tables from the polynomials too in float32 (the fit's
    // derivative error, about the degree squared times the fit tolerance of
    // 1e-9, stays far below float32 rounding); float64 evaluates them.
    constexpr bool POLY_D = sizeof(R) == 4;
    if (poly && (!GRAD || POLY_D)) {
        // the fitted polynomials: a short body, unrolled, so that w stays in
        // registers.  The window is even, so tap 2m - 1 - t at v is tap t at
        // -v: both come from the even and odd parts of tap t's polynomial.
#pragma unroll
        for (int dim = 0; dim < 3; ++dim) {
            const double v = 2.0 * u[dim] - 1.0, v2 = v * v;
#pragma unroll
            for (int t = 0; t < m; ++t) {
                const double *c = poly + t * NC;
                double ev = c[(NC - 1) & ~1], od = c[(NC - 2) | 1];
#pragma unroll
                for (int k = ((NC - 1) & ~1) - 2; k >= 0; k -= 2) ev = fma(ev, v2, c[k]);
#pragma unroll
                for (int k = ((NC - 2) | 1) - 2; k >= 1; k -= 2) od = fma(od, v2, c[k]);
                w[dim * M2 + t] = (R)fma(v, od, ev);
                w[dim * M2 + M2 - 1 - t] = (R)fma(-v, od, ev);
                if constexpr (GRAD) {
                    // P(v) approximates phi(u + m - 1 - t) with v = 2u - 1, so
                    // phi' there is 2 P'(v).  P'(v) = A(v^2) + v B(v^2): A
                    // sums k c_k v^(k-1) over odd k, B over even k >= 2.  Tap
                    // 2m - 1 - t is P(-v), whose phi' is -2 P'(-v).
                    constexpr int KA = ((NC - 1) & 1) ? NC - 1 : NC - 2;  // top odd k
                    constexpr int KB = ((NC - 1) & 1) ? NC - 2 : NC - 1;  // top even k
                    double a = KA * c[KA], b = KB * c[KB];
#pragma unroll
                    for (int k = KA - 2; k >= 1; k -= 2) a = fma(a, v2, k * c[k]);
#pragma unroll
                    for (int k = KB - 2; k >= 2; k -= 2) b = fma(b, v2, k * c[k]);
                    const double s = 2.0 * (double)n[dim];
                    dw[dim * M2 + t] = (R)(s * fma(v, b, a));
                    dw[dim * M2 + M2 - 1 - t] = (R)(-s * fma(-v, b, a));
                }
            }
            if (dim < flat) {
#pragma unroll
                for (int t = 0; t < M2; ++t) {
                    w[dim * M2 + t] = t == m - 1 ? R(1) : R(0);
                    if constexpr (GRAD) dw[dim * M2 + t] = R(0);
                }
            }
        }
    } else {
        // direct evaluation (and the derivatives): a loop too large to
        // unroll, into arrays of its own, then copied with fixed indices (an
        // array indexed at run time would leave w in scratch memory for
        // every path)
        constexpr int NW = 3 * M2;
        R ws[NW], dws[GRAD ? NW : 1];
        for (int dim = 0; dim < 3; ++dim) {
            for (int t = 0; t < M2; ++t) {
                const double dist = u[dim] + (double)(m - 1 - t);
                double ph = 0.0, dph = 0.0;
                win_eval(wp, dist, &ph, GRAD ? &dph : nullptr);
                ws[dim * M2 + t] = (R)(poly ? horner<NC>(poly + t * NC, 2.0 * u[dim] - 1.0) : ph);
                if constexpr (GRAD) dws[dim * M2 + t] = (R)((double)n[dim] * dph);
                if (dim < flat) {
                    ws[dim * M2 + t] = t == m - 1 ? R(1) : R(0);
                    if constexpr (GRAD) dws[dim * M2 + t] = R(0);
                }
            }
        }
#pragma unroll
        for (int i = 0; i < NW; ++i) {
            w[i] = ws[i];
            if constexpr (GRAD) dw[i] = dws[i];
        }
    }
    // dim 0 into slot order, slot s = (tap + rot) mod 2m: a rotation by rot
    // composed of conditional rotations by 1, 2, 4, ... (constant indices).
    // The box method keeps tap order.
    if (nb0) rot = 0;
#pragma unroll
    for (int k = 1; k < M2; k <<= 1) {
        if (rot & k) {
            R tmp[M2], dtmp[GRAD ? M2 : 1];
#pragma unroll
            for (int s = 0; s < M2; ++s) {
                tmp[s] = w[(s - k + M2) % M2];
                if constexpr (GRAD) dtmp[s] = dw[(s - k + M2) % M2];
            }
#pragma unroll
            for (int s = 0; s < M2; ++s) {
                w[s] = tmp[s];
                if constexpr (GRAD) dw[s] = dtmp[s];
            }
        }
    }
    // blocks of lines (line method): dim 2 in lane order, slot x = (tap +
    // j) mod 2m for the point's line j in its block, so that the lane of
    // block column x (which receives tap (x - j) mod 2m) reads a fixed slot
    if (block_w(M2) > 1 && !nb0) {
        const int jl = c[2] & (block_w(M2) - 1);  // (c2 mod T) mod BW, BW dividing T
#pragma unroll
        for (int k = 1; k < M2; k <<= 1) {
            if (jl & k) {
                R tmp[M2], dtmp[GRAD ? M2 : 1];
#pragma unroll
                for (int s = 0; s < M2; ++s) {
                    tmp[s] = w[2 * M2 + (s - k + M2) % M2];
                    if constexpr (GRAD) dtmp[s] = dw[2 * M2 + (s - k + M2) % M2];
                }
#pragma unroll
                for (int s = 0; s < M2; ++s) {
                    w[2 * M2 + s] = tmp[s];
                    if constexpr (GRAD) dw[2 * M2 + s] = dtmp[s];
                }
            }
        }
    }
    head = nb0 ? make_int2(c[0], (c[1] << kBoxCellBits) | c[2]) : make_int2(c[0], c[2] & (block_w(M2) - 1));
    return pos;
}

// One thread per point, each storing its own record (gradient plans, whose
// records carry the derivative tables too).
template <typename R, int M2, bool GRAD>
__global__ __launch_bounds__(256) void k_bin_scatter(const double *__restrict__ xd, const float *__restrict__ xf,
                                                     long long M, long long poff, int n0, int n1, int n2, int T,
                                                     int ntx, const int *__restrict__ cell_start,
                                                     const int *__restrict__ rank, int *__restrict__ perm,
                                                     int *__restrict__ ipos, unsigned char *__restrict__ rec,
                                                     size_t rec_bytes, WindowParams wp,
                                                     const double *__restrict__ poly, int flat, int nb0, int nb1,
                                                     int nb2, const int *__restrict__ fixed_pos)
{
    constexpr int NW = 3 * M2;
    static_assert((NW * sizeof(R)) % 8 == 0, "window block is a whole number of 8-byte units");
    const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    R w[NW];
    R dw[GRAD ? NW : 1];
    int2 head;
    const long long pos = scatter_point<R, M2, GRAD>(j, xd, xf, poff, n0, n1, n2, T, ntx, cell_start, rank, perm,
                                                     ipos, wp, poly, flat, nb0, nb1, nb2, fixed_pos, w, dw, head);
    unsigned char *rp = rec + pos * rec_bytes;
    store_block<NW * sizeof(R)>(rp, w);
    *reinterpret_cast<int2 *>(rp + rec_off_pz(M2, sizeof(R))) = head;
    if constexpr (GRAD) store_block<NW * sizeof(R)>(rp + rec_prefix(M2, sizeof(R)), dw);
}

// Records without derivative tables: each wavefront assembles its 64
// records in LDS, then stores them unit by unit, consecutive lanes on
// consecutive 16-byte units, so that a store instruction writes a few whole
// records instead of one 16-byte piece of 64 records.  The value slot is
// left zero (the sweeps that stage records fill it per call).
template <typename R, int M2>
__global__ __launch_bounds__(64) void k_bin_scatter_lds(const double *__restrict__ xd, const float *__restrict__ xf,
                                                        long long M, long long poff, int n0, int n1, int n2, int T,
                                                        int ntx, const int *__restrict__ cell_start,
                                                        const int *__restrict__ rank, int *__restrict__ perm,
                                                        int *__restrict__ ipos, unsigned char *__restrict__ rec,
                                                        size_t rec_bytes, WindowParams wp,
                                                        const double *__restrict__ poly, int flat, int nb0, int nb1,
                                                        int nb2, const int *__restrict__ fixed_pos)
{
    constexpr int NW = 3 * M2;
    constexpr int RB = (int)rec_prefix(M2, sizeof(R));  // record bytes staged
    constexpr int U = RB / 16;
    static_assert(RB % 16 == 0 && (NW * sizeof(R)) % 8 == 0, "records of whole 16-byte units");
    extern __shared__ uint4 sm[];  // 64 records, then 64 positions
    int *spos = reinterpret_cast<int *>(sm + 64 * U);
    const int lane = threadIdx.x;
    const long long j0 = (long long)blockIdx.x * 64;
    const long long j = j0 + lane;
    if (j < M) {
        R w[NW];
        R dw[1];
        int2 head;
        const long long pos = scatter_point<R, M2, false>(j, xd, xf, poff, n0, n1, n2, T, ntx, cell_start, rank,
                                                          perm, ipos, wp, poly, flat, nb0, nb1, nb2, fixed_pos, w,
                                                          dw, head);
        uint4 *lp = sm + lane * U;
        constexpr int NU32 = NW * (int)sizeof(R) / 4;  // words of the window tables
        unsigned wv[NU32];
        __builtin_memcpy(wv, w, sizeof(wv));  // (a copy: no access through a pointer of another type)
        // words NU32 .. : value slot (zero), header, padding (zero)
        unsigned tail[4 * U - NU32];
#pragma unroll
        for (int i = 0; i < 4 * U - NU32; ++i) tail[i] = 0u;
        constexpr int HW = (int)rec_off_pz(M2, sizeof(R)) / 4 - NU32;  // header word in tail
        tail[HW] = (unsigned)head.x;
        tail[HW + 1] = (unsigned)head.y;
#pragma unroll
        for (int k = 0; k < U; ++k) {
            unsigned v[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int wi = 4 * k + i;
                v[i] = wi < NU32 ? wv[wi] : tail[wi - NU32];
            }
            lp[k] = make_uint4(v[0], v[1], v[2], v[3]);
        }
        spos[lane] = (int)pos;
    }
    __syncthreads();
    const int nvalid = (int)(M - j0 < 64 ? M - j0 : 64);
    for (int u = lane; u < nvalid * U; u += 64) {
        const int r = u / U, k = u - r * U;
        *reinterpret_cast<uint4 *>(rec + (size_t)spos[r] * rec_bytes + 16 * k) = sm[r * U + k];
    }
}

// ---------------------------------------------------------------------------
// Exclusive prefix sum (in place) over int counts, in blocks of 4096: a
// reduce pass writes each block's total; the scan pass then scans each block
// from the sum of the totals before it.  Up to kScanDirect blocks, each block
// adds those totals itself (at most 32 loads per thread), so the scan is two
// launches; longer arrays scan the totals recursively first.
constexpr int kScanThreads = 256;
constexpr int kScanPer = 16;                         // 4 int4 per thread
constexpr int kScanBlock = kScanThreads * kScanPer;  // 4096 elements
constexpr long long kScanDirect = 8192;

// Exclusive scan of one int per thread over the 256-thread block; *total =
// the block's sum.  sh: 4 ints of LDS.
__device__ inline int scan_block256(int v, int *sh, int *total)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) sh[w] = x;
    __syncthreads();
    int pre = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < kScanThreads / 64; ++k) {
        const int t = sh[k];
        pre += k < w ? t : 0;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return pre + x - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const int *__restrict__ data, long long n,
                                                              int *__restrict__ sums)
{
    __shared__ int sh[kScanThreads / 64];
    const int4 *d4 = reinterpret_cast<const int4 *>(data);
    const long long n4 = n / 4;
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanPer / 4; ++k) {
        const long long i4 = (long long)blockIdx.x * (kScanBlock / 4) + k * kScanThreads + threadIdx.x;
        if (i4 < n4) {
            const int4 v = d4[i4];
            s += v.x + v.y + v.z + v.w;
        } else if (i4 == n4) {
            for (long long e = n4 * 4; e < n; ++e) s += data[e];
        }
    }
    int total;
    scan_block256(s, sh, &total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// offs: block totals (direct: their prefix is summed here) or, when
// !direct, already-scanned block offsets; null for a single block.
__global__ __launch_bounds__(kScanThreads) void k_scan_apply(int *__restrict__ data, long long n,
                                                             const int *__restrict__ offs, int direct)
{
    __shared__ int sh[kScanThreads / 64];
    int base = 0;
    if (offs) {
        if (direct) {
            int o = 0;
            for (int i = threadIdx.x; i < (int)blockIdx.x; i += kScanThreads) o += offs[i];
            scan_block256(o, sh, &base);
        } else {
            base = offs[blockIdx.x];
        }
    }
    const long long e0 = (long long)blockIdx.x * kScanBlock + (long long)threadIdx.x * kScanPer;
    int v[kScanPer];
    const bool full = e0 + kScanPer <= n;
    if (full) {
#pragma unroll
        for (int k = 0; k < kScanPer / 4; ++k) {
            const int4 q = reinterpret_cast<const int4 *>(data + e0)[k];
            v[4 * k] = q.x;
            v[4 * k + 1] = q.y;
            v[4 * k + 2] = q.z;
            v[4 * k + 3] = q.w;
        }
    } else {
#pragma unroll
        for (int i = 0; i < kScanPer; ++i) v[i] = e0 + i < n ? data[e0 + i] : 0;
    }
    int s = 0;
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) s += v[i];
    int total;
    int run = base + scan_block256(s, sh, &total);
#pragma unroll
    for (int i = 0; i < kScanPer; ++i) {
        const int c = v[i];
        v[i] = run;
        run += c;
    }
    if (full) {
#pragma unroll
        for (int k = 0; k < kScanPer / 4; ++k)
            reinterpret_cast<int4 *>(data + e0)[k] = make_int4(v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]);
    } else {
#pragma unroll
        for (int i = 0; i < kScanPer; ++i)
            if (e0 + i < n) data[e0 + i] = v[i];
    }
}

// data must be 16-byte aligned; tmp holds nb + nb / 2048 + 64 ints.
hipError_t launch_scan(int *data, long long n, int *tmp, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const long long nb = (n + kScanBlock - 1) / kScanBlock;
    if (nb <= 1) {
        hipLaunchKernelGGL(k_scan_apply, dim3(1), dim3(kScanThreads), 0, s, data, n, (const int *)nullptr, 0);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanThreads), 0, s, data, n, tmp);
    const bool direct = nb <= kScanDirect;
    if (!direct) {
        hipError_t e = launch_scan(tmp, nb, tmp + nb, s);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kScanThreads), 0, s, data, n, (const int *)tmp,
                       direct ? 1 : 0);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
hipError_t launch_bin_count(const double *x, const float *xf32, long long M, const Xform &X, int T, int BW,
                            int flat, int *counts, int *rank, int *err, double *xs_out, int *keys_out,
                            hipStream_t s)
{
    if (M <= 0) return hipSuccess;
    const unsigned nb = (unsigned)((M + 255) / 256);
    if (x)
        hipLaunchKernelGGL(k_bin_count<double>, dim3(nb), dim3(256), 0, s, x, M, X.n[0], X.n[1], X.n[2], T,
                           X.ntx, BW, flat, X.nbox[0], X.nbox[1], X.nbox[2], counts, rank, err, xs_out, keys_out);
    else
        hipLaunchKernelGGL(k_bin_count<float>, dim3(nb), dim3(256), 0, s, xf32, M, X.n[0], X.n[1], X.n[2], T,
                           X.ntx, BW, flat, X.nbox[0], X.nbox[1], X.nbox[2], counts, rank, err, xs_out, keys_out);
    return hipGetLastError();
}

template <typename R, int M2>
static void scatter_m(const double *x, const float *xf32, long long M, const Xform &X, int T,
                      const int *cell_start, const int *rank, int *perm, int *ipos, unsigned char *rec,
                      size_t rec_bytes, const WindowParams &wp, const double *poly, bool grad, const int *fixed_pos,
                      hipStream_t s)
{
    if (!grad) {
        constexpr size_t lds = 64 * rec_prefix(M2, sizeof(R)) + 64 * 4;
        const unsigned nb = (unsigned)((M + 63) / 64);
        auto kl = k_bin_scatter_lds<R, M2>;
        hipLaunchKernelGGL(kl, dim3(nb), dim3(64), lds, s, x, xf32, M, X.poff, X.n[0],
                           X.n[1], X.n[2], T, X.ntx, cell_start, rank, perm, ipos, rec, rec_bytes, wp, poly, X.flat,
                           X.nbox[0], X.nbox[1], X.nbox[2], fixed_pos);
        return;
    }
    const unsigned nb = (unsigned)((M + 255) / 256);
    auto kg = k_bin_scatter<R, M2, true>;
    hipLaunchKernelGGL(kg, dim3(nb), dim3(256), 0, s, x, xf32, M, X.poff, X.n[0], X.n[1],
                       X.n[2], T, X.ntx, cell_start, rank, perm, ipos, rec, rec_bytes, wp, poly, X.flat, X.nbox[0],
                       X.nbox[1], X.nbox[2], fixed_pos);
}

template <typename R>
hipError_t launch_bin_scatter(const double *x, const float *xf32, long long M, const Xform &X, int T, int m,
                              const WindowParams &wp, const double *poly, const int *cell_start, const int *rank,
                              int *perm, int *ipos, unsigned char *rec, size_t rec_bytes, bool grad,
                              const int *fixed_pos, hipStream_t s)
{
    if (M <= 0) return hipSuccess;
    switch (m) {
#define HPNFFT_SCATTER_CASE(MM) \
    case MM: scatter_m<R, 2 * MM>(x, xf32, M, X, T, cell_start, rank, perm, ipos, rec, rec_bytes, wp, poly, grad, fixed_pos, s); break;
        HPNFFT_SCATTER_CASE(1)
        HPNFFT_SCATTER_CASE(2)
        HPNFFT_SCATTER_CASE(3)
        HPNFFT_SCATTER_CASE(4)
        HPNFFT_SCATTER_CASE(5)
        HPNFFT_SCATTER_CASE(6)
        HPNFFT_SCATTER_CASE(7)
        HPNFFT_SCATTER_CASE(8)
        HPNFFT_SCATTER_CASE(9)
        HPNFFT_SCATTER_CASE(10)
        HPNFFT_SCATTER_CASE(11)
        HPNFFT_SCATTER_CASE(12)
        HPNFFT_SCATTER_CASE(13)
        HPNFFT_SCATTER_CASE(14)
        HPNFFT_SCATTER_CASE(15)
#undef HPNFFT_SCATTER_CASE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template hipError_t launch_bin_scatter<double>(const double *, const float *, long long, const Xform &, int, int,
                                               const WindowParams &, const double *, const int *, const int *, int *, int *,
                                               unsigned char *, size_t, bool, const int *, hipStream_t);
template hipError_t launch_bin_scatter<float>(const double *, const float *, long long, const Xform &, int, int,
                                              const WindowParams &, const double *, const int *, const int *, int *, int *,
                                              unsigned char *, size_t, bool, const int *, hipStream_t);

}  // namespace hpnfft
