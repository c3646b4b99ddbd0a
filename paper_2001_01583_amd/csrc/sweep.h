// Spreading (the Spreading step of Algorithm 2, Section 3) and interpolation
// (the Interpolating step of Algorithm 5) on gfx950.
//
// The paper assigns one thread per point and adds every window tap to the
// grid with an atomic operation.  Here points are sorted into runs: a z-line
// (fixed cells in dims 1 and 2) or, for 2m = 8, a block of 8 z-lines adjacent
// along dim 2, each run ordered by plane along dim 0.  A work item is a tile
// of T x T z-lines restricted to a slab of Zs planes along dim 0.
//
// Per work item a workgroup
//   1. lists the item's runs: for every run up to three contiguous ranges of
//      sorted points (the periodic images whose taps reach the slab), and
//      numbers their points 0 .. S-1 in run order;
//   2. for each chunk of `cap` of those points, copies the points' records
//      (window weights, value, plane index) into LDS with all threads at once
//      (coalesced 16-byte copies; the next chunk loads into registers while
//      the current one is swept);
//   3. sweeps the chunk, one wavefront per task (a run, or for blocks an
//      equal range of the chunk's points).  Lane <-> one (dy, dx) tap row of
//      a line's (2m)^2 rows; in a block, lane (dy, xm) owns the tile columns
//      x0 + xm and x0 + xm + 8 of tap row dy, which between them receive
//      every tap of row dy from all 8 lines.  Along dim 0 each owned row has
//      a register window of 2m complex values, slot s holding plane q with
//      q = s (mod 2m).  The sweep is plane-major: the plane loop is unrolled
//      2m times, so a plane's slot is a compile-time constant; the points
//      whose window starts at plane p are added, then plane p leaves the
//      window (spread: one LDS add per owned row).  Weights along dim 0 are
//      stored pre-rotated per point to slot order;
//   4. flushes the LDS tile (the slab's planes with a halo of 2m-1 cells in
//      dims 1 and 2) to the grid with one atomic add per cell.
// Interpolation loads the tile from the grid, slides the same register
// window (loading a plane when it enters) and reduces the (2m)^2 row partials
// of each point across the wavefront with swap/DPP halving steps.
//
// Work items come from a device queue (one atomic per item) so heavy tiles
// and uneven batches balance across the compute units.
#pragma once

#include <algorithm>

#include "internal.h"
#include "wave_reduce.h"

namespace hpnfft {

// Value known to be equal on all lanes of the wavefront, moved to a scalar
// register so that branches on it are scalar branches.
__device__ inline int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

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

// Compensated float adds into K LDS cells at once (the real and imaginary
// parts of the lane's tile values, kept in separate arrays), each cell holding
// (sum, compensation) as one 64-bit word: TwoSum (Knuth) of the stored sum and
// v gives the new sum and its exact rounding error, which joins the
// compensation; each pair is published with a 64-bit compare-and-swap.  The K
// reads, then the K swaps are issued back to back, so a retire costs two LDS
// round trips whatever K is.  The initial read is only a guess: a swap that
// finds another value (a wavefront of the same workgroup added to the cell in
// between) is retried from the value it found.  A lane with nothing to add
// for cell k passes ok[k] = false and c[k] = a cell that nobody changes: it
// swaps that cell's value with itself.
// (gfx950's native LDS float32 atomic add is about 13x slower than this.)
__device__ __forceinline__ unsigned long long twosum_pair(unsigned long long old, float v)
{
    const float sm = __uint_as_float((unsigned int)old);
    const float cp = __uint_as_float((unsigned int)(old >> 32));
    const float t = sm + v;
    const float bp = t - sm;
    const float e = (sm - (t - bp)) + (v - bp);
    return (unsigned long long)__float_as_uint(t) | ((unsigned long long)__float_as_uint(cp + e) << 32);
}

template <int K>
__device__ __forceinline__ void lds_add_comp(unsigned long long *const (&c)[K], const float (&v)[K],
                                             const bool (&ok)[K])
{
    unsigned long long o[K], pr[K];
#pragma unroll
    for (int k = 0; k < K; ++k) o[k] = *c[k];
    unsigned long long nw[K];
#pragma unroll
    for (int k = 0; k < K; ++k) nw[k] = ok[k] ? twosum_pair(o[k], v[k]) : o[k];
    // keep the K swaps together: they then share one wait
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < K; ++k) pr[k] = atomicCAS(c[k], o[k], nw[k]);
    __builtin_amdgcn_sched_barrier(0);
    bool miss = false;
#pragma unroll
    for (int k = 0; k < K; ++k) miss |= pr[k] != o[k];
    if (__builtin_expect(__any(miss), 0)) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            while (pr[k] != o[k]) {
                o[k] = pr[k];
                pr[k] = atomicCAS(c[k], o[k], ok[k] ? twosum_pair(o[k], v[k]) : o[k]);
            }
        }
    }
}

// Exclusive scan of one int per thread over the workgroup (<= 1024 threads);
// sh: 32 ints of LDS.  Contains barriers: call from all threads.
__device__ inline int block_excl_scan(int v, int *sh, int *total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) sh[wave] = x;
    __syncthreads();
    if (wave == 0) {
        int w = lane < nw ? sh[lane] : 0;
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) {
            int y = __shfl_up(w, o, 64);
            if (lane >= o) w += y;
        }
        if (lane < nw) sh[16 + lane] = w;
    }
    __syncthreads();
    int before = wave > 0 ? sh[16 + wave - 1] : 0;
    *total = sh[16 + nw - 1];
    __syncthreads();
    return before + x - v;
}

// Largest r in [0, nr) with soff[r] <= v (soff non-decreasing, soff[nr] > v).
__device__ inline int find_run(const int *soff, int nr, int v)
{
    int lo = 0, hi = nr;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (soff[mid] <= v) lo = mid;
        else hi = mid;
    }
    return lo;
}

__device__ inline int next_item(int *queue, int *s_item)
{
    __syncthreads();
    if (threadIdx.x == 0) *s_item = atomicAdd(queue, 1);
    __syncthreads();
    return *s_item;
}

// The work-queue counter clears itself: the last workgroup to finish resets
// it (and the finish count two words on) to zero, so the next launch needs
// no clearing, and a captured graph no memset.  Call from all threads after
// the item loop (whose last next_item ends with a barrier): by then this
// workgroup has taken its last item.
__device__ inline void release_queue(int *queue)
{
    if (threadIdx.x == 0) {
        const int done = atomicAdd(queue + 2, 1);
        if (done == (int)gridDim.x - 1) {
            atomicExch(queue, 0);
            atomicExch(queue + 2, 0);
        }
    }
}

// Geometry of one work item.
struct ItemGeom {
    int n0, n1, n2, X0, Y0, z0, zs, ry0, nrows, lb, le, tile;
    long long poff, key_off;
};

__device__ inline ItemGeom item_geom(const SItem &W, const Xform &X, int T, int Zs, int M2)
{
    ItemGeom g;
    g.n0 = X.n[0];
    g.n1 = X.n[1];
    g.n2 = X.n[2];
    g.X0 = (W.tile % X.ntx) * T;
    g.Y0 = (W.tile / X.ntx) * T;
    g.z0 = W.slab * Zs;
    g.zs = min(Zs, g.n0 - g.z0);
    const int LPR = T / block_w(M2);  // runs per tile row
    g.ry0 = W.lb / LPR;
    g.nrows = (W.le - 1) / LPR + M2 - g.ry0;
    g.lb = W.lb;
    g.le = W.le;
    g.tile = W.tile;
    g.poff = X.poff;
    g.key_off = X.key_off;
    return g;
}

// Step 1: run list of the item.  A line here is one sorted run: a block of
// BW z-lines (see block_w).  Run r = 3 * (line - lb) + (segment + 1);
// run_p0[r] = first sorted point, run_soff = exclusive prefix of run sizes
// (run_soff[nr] = S).  Returns S.  Contains barriers.
template <int M2>
__device__ inline int build_runs(const ItemGeom &g, int T, const int *__restrict__ cell_start, int *run_p0,
                                 int *run_soff, int *sh)
{
    constexpr int m = M2 / 2;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int nr = 3 * (g.le - g.lb);
    const int k = (nr + nthr - 1) / nthr;
    int local = 0;
    for (int i = 0; i < k; ++i) {
        int r = tid * k + i;
        if (r >= nr) break;
        constexpr int BW = block_w(M2);
        const int LPR = T / BW;
        int li = g.lb + r / 3, U = (r % 3 - 1) * g.n0;
        int ly = li / LPR, lx = (li % LPR) * BW;
        int cnt = 0, p0 = 0;
        if (g.Y0 + ly < g.n1 && g.X0 + lx < g.n2) {
            int a, b;
            seg_range(U, g.z0, g.zs, m, g.n0, &a, &b);
            if (a <= b) {
                const int *cs = cell_start + g.key_off + ((long long)g.tile * (T * T / BW) + li) * g.n0 * BW;
                p0 = cs[a * BW];
                cnt = cs[(b + 1) * BW] - p0;
            }
        }
        run_p0[r] = (int)(g.poff + p0);
        run_soff[r] = cnt;
        local += cnt;
    }
    int total;
    int base = block_excl_scan(local, sh, &total);
    for (int i = 0; i < k; ++i) {
        int r = tid * k + i;
        if (r >= nr) break;
        int c = run_soff[r];
        run_soff[r] = base;
        base += c;
    }
    if (tid == 0) run_soff[nr] = total;
    __syncthreads();
    return total;
}

// Step 2: chunks of the item's point stream are staged into LDS.  While a
// chunk is swept, the next chunk's records are already loading into
// registers (up to PF 16-byte units per thread; any remainder is copied
// after the sweep), so HBM latency overlaps the sweep.

// 16-byte unit of the record copies (a native vector type, so that the
// prefetch array is kept in registers).
typedef unsigned int v4u __attribute__((ext_vector_type(4)));

// Window base of a staged point: first tap plane along dim 0 plus 2m (so
// that it is never negative), as a wave-uniform value.
constexpr int kNoPlane = 0x7fffffff;
__device__ inline int plane_of(const v4u *stage, int sl, int st16, int off_pz, int m)
{
    return uni(reinterpret_cast<const int *>(stage + sl * st16)[off_pz]) + m + 1;
}

// Plane index and line offset of a staged point (one 8-byte read), raw.
__device__ inline int2 head_of(const v4u *stage, int sl, int st16, int off_pz)
{
    return *reinterpret_cast<const int2 *>(reinterpret_cast<const int *>(stage + sl * st16) + off_pz);
}

// slot -> sorted point map of the chunk [cs, cs + cnt).  No barrier.
__device__ inline void chunk_slots(int cs, int cnt, int nr, const int *run_p0, const int *run_soff, int *slot_p)
{
    for (int s = threadIdx.x; s < cnt; s += blockDim.x) {
        int v = cs + s;
        int r = find_run(run_soff, nr, v);
        slot_p[s] = run_p0[r] + (v - run_soff[r]);
    }
}

// The spread takes each point's value from the values in sorted order (fs,
// written per call) rather than from its record: 16-byte unit uf of a staged
// record receives it, at word wf (float: 2 words, double: the whole unit).
struct ValueSlot {
    const void *fs;  // null: stage the records as they are
    int uf, wf;
};
template <typename R>
__device__ inline v4u with_value(v4u v, const ValueSlot &vs, long long sp)
{
    if constexpr (sizeof(R) == 8) {
        return reinterpret_cast<const v4u *>(vs.fs)[sp];
    } else {
        const uint2 q = reinterpret_cast<const uint2 *>(vs.fs)[sp];
        if (vs.wf == 0) {
            v.x = q.x;
            v.y = q.y;
        } else {
            v.z = q.x;
            v.w = q.y;
        }
        return v;
    }
}

template <int PF, typename R>
__device__ inline void chunk_fetch(int cnt, const int *slot_p, int st16, const v4u *__restrict__ rec, int rs16,
                                   const ValueSlot &vs, v4u (&reg)[PF])
{
    // every thread loads PF units; indices past the chunk reload unit 0 (the
    // chunk is never empty), so the loads need no branch and the array stays
    // in registers
    const int tot = cnt * st16;
#pragma unroll
    for (int k = 0; k < PF; ++k) {
        int e = threadIdx.x + k * blockDim.x;
        e = e < tot ? e : 0;
        const int sl = e / st16, u = e - sl * st16;
        const long long sp = slot_p[sl];
        v4u v = rec[sp * rs16 + u];
        if (vs.fs && u == vs.uf) v = with_value<R>(v, vs, sp);
        reg[k] = v;
    }
}

template <int PF, typename R>
__device__ inline void chunk_store(int cnt, const int *slot_p, int st16, const v4u *__restrict__ rec, int rs16,
                                   const ValueSlot &vs, const v4u (&reg)[PF], v4u *stage)
{
    const int tot = cnt * st16;
#pragma unroll
    for (int k = 0; k < PF; ++k) {
        int e = threadIdx.x + k * blockDim.x;
        if (e < tot) stage[e] = reg[k];
    }
    for (int e = threadIdx.x + PF * blockDim.x; e < tot; e += blockDim.x) {
        const int sl = e / st16, u = e - sl * st16;
        const long long sp = slot_p[sl];
        v4u v = rec[sp * rs16 + u];
        if (vs.fs && u == vs.uf) v = with_value<R>(v, vs, sp);
        stage[e] = v;
    }
}

// ---------------------------------------------------------------------------
// Spread.  COMP: float path with per-bin compensated sums: every LDS tile
// cell is a (sum, compensation) pair updated by lds_add_comp.  The float64
// path adds with the native LDS float64 atomic.
template <typename R, int M2, bool COMP>
__global__ __launch_bounds__(spread_max_threads(sizeof(R), M2)) void k_spread(const Xform *__restrict__ xfs,
                                                 const SItem *__restrict__ items, int nitems,
                                                 int *__restrict__ queue, int T, int Zs, int cap,
                                                 const v4u *__restrict__ rec, int rs16,
                                                 const R *__restrict__ fs, const int *__restrict__ cell_start)
{
    constexpr int m = M2 / 2;
    constexpr int ROWS = M2 * M2;
    constexpr int NRG = (ROWS + 63) / 64;
    constexpr int ST16 = (int)(rec_prefix(M2, sizeof(R)) / 16);
    constexpr int OFF_F = (int)(rec_off_f(M2, sizeof(R)) / sizeof(R));
    const ValueSlot vs{fs, (int)(rec_off_f(M2, sizeof(R)) / 16), (int)(rec_off_f(M2, sizeof(R)) % 16 / 4)};
    static_assert(rec_off_f(M2, sizeof(R)) % 8 == 0 && rec_off_f(M2, sizeof(R)) % 16 + 2 * sizeof(R) <= 16,
                  "the value lies within one 16-byte unit of the record");
    constexpr int OFF_PZ = (int)(rec_off_pz(M2, sizeof(R)) / 4);
    static_assert(rec_off_xr(M2, sizeof(R)) == rec_off_pz(M2, sizeof(R)) + 4 && rec_off_pz(M2, sizeof(R)) % 8 == 0,
                  "head_of reads the plane index and line offset as one int2");
    constexpr int BW = block_w(M2);
    constexpr int NW = BW > 1 ? 2 : 1;  // tile rows per lane
    static_assert(BW == 1 || BW * BW == 64, "a blocked sweep maps (dy, xm) onto the 64 lanes");
    extern __shared__ uint4 smem16[];
    unsigned char *smem = reinterpret_cast<unsigned char *>(smem16);
    __shared__ int s_item;
    const LdsLayout LL = lds_layout(T, Zs, M2, sizeof(R), 0, COMP, cap);
    const int LPR = T / BW;  // runs (blocks of lines) per tile row
    const int P = T + M2 - 1;
    // tile: real parts [Zs][P][pitch] of 8-byte cells, then imaginary parts
    const int pitch = spread_pitch(T, M2);
    const int plane = P * pitch;
    const int im_off = Zs * plane;  // LDS indices fit in 32 bits
    R *acc = reinterpret_cast<R *>(smem + LL.tile);
    unsigned long long *pairs = reinterpret_cast<unsigned long long *>(smem + LL.tile);
    v4u *stage = reinterpret_cast<v4u *>(smem + LL.stage);
    int *slot_a = reinterpret_cast<int *>(smem + LL.slot_p);
    int *slot_b = slot_a + cap;
    int *run_p0 = reinterpret_cast<int *>(smem + LL.run_p0);
    int *run_soff = reinterpret_cast<int *>(smem + LL.run_soff);
    int *sh = reinterpret_cast<int *>(smem + LL.sh);
    unsigned long long *still = reinterpret_cast<unsigned long long *>(smem + LL.sh + 32 * 4);
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int wave = uni(tid >> 6), lane = tid & 63, nwaves = nthr >> 6;
    constexpr int PF = (sizeof(R) == 8 && M2 >= 12) ? 2 : 4;

    for (int it = next_item(queue, &s_item); it < nitems; it = next_item(queue, &s_item)) {
        const ItemGeom g = item_geom(items[it], xfs[items[it].xf], T, Zs, M2);
        const int nz = g.zs * g.nrows * P;
        for (int i = tid; i < nz; i += nthr) {
            int z = i / (g.nrows * P), rem = i - z * g.nrows * P;
            const int o = z * plane + (g.ry0 + rem / P) * pitch + rem % P;
            if (COMP) {
                pairs[o] = 0ull;
                pairs[o + im_off] = 0ull;
            } else {
                acc[o] = R(0);
                acc[o + im_off] = R(0);
            }
        }
        const int nr = 3 * (g.le - g.lb);
        const int S = build_runs<M2>(g, T, cell_start, run_p0, run_soff, sh);

        const int nch = (S + cap - 1) / cap;
        v4u reg[PF];
        if (nch > 0) {
            const int c0n = min(cap, S);
            chunk_slots(0, c0n, nr, run_p0, run_soff, slot_a);
            __syncthreads();
            chunk_fetch<PF, R>(c0n, slot_a, ST16, rec, rs16, vs, reg);
            chunk_store<PF, R>(c0n, slot_a, ST16, rec, rs16, vs, reg, stage);
            __syncthreads();
        }
        for (int ch = 0; ch < nch; ++ch) {
            const int cs = ch * cap;
            const int cnt = min(cap, S - cs);
            int *slot_n = (ch & 1) ? slot_a : slot_b;
            const bool more = ch + 1 < nch;
            const int cntn = more ? min(cap, S - cs - cap) : 0;
            if (more) {
                chunk_slots(cs + cap, cntn, nr, run_p0, run_soff, slot_n);
                __syncthreads();
                chunk_fetch<PF, R>(cntn, slot_n, ST16, rec, rs16, vs, reg);
            }
            // Tasks (times row groups): blocks of lines hold long runs, so
            // their tasks are equal ranges of the chunk's points (one per
            // wavefront: a run cut into more pieces re-adds the 2m - 1 planes
            // its window carries over each cut), each sweeping the run pieces
            // it covers; single
            // lines hold short runs and take one run per task.
            const int r_lo = uni(find_run(run_soff, nr, cs));
            const int r_hi = uni(find_run(run_soff, nr, cs + cnt - 1));
            const int piece = max(16, (cnt + nwaves - 1) / nwaves);
            const int ntask = (BW > 1 ? (cnt + piece - 1) / piece : r_hi - r_lo + 1) * NRG;
            for (int task = wave; task < ntask; task += nwaves) {
              const int rg = task % NRG;
              int lo = cs, hi = cs + cnt, rf = r_lo + task / NRG;
              if (BW > 1) {
                  lo = cs + (task / NRG) * piece;
                  hi = min(cs + cnt, lo + piece);
                  rf = uni(find_run(run_soff, nr, lo));
              }
              for (int r = rf; r < nr && uni(run_soff[r]) < hi && (BW > 1 || r == rf); ++r) {
                const int a = uni(max(run_soff[r], lo) - cs);
                const int b = uni(min(run_soff[r + 1], hi) - cs);
                if (a >= b) continue;
                const int li = g.lb + r / 3;
                const int U = (r % 3 - 1) * g.n0;
                const int ly = li / LPR, lx = (li % LPR) * BW;  // the run's first line
                const int row = rg * 64 + lane;
                const bool active = ROWS % 64 == 0 || row < ROWS;
                // Rows of the LDS tile this lane owns.  Single lines: tap
                // row (dy, dx) of the line.  Blocks of 8 lines (2m = 8):
                // lane (dy, xm) owns columns lx + xm and lx + xm + 8 of tap
                // row dy; a point on line lx + j reaches column lx + xm
                // (dx = xm - j) when xm >= j, else lx + xm + 8.
                const int dy = active ? row / (BW > 1 ? BW : M2) : 0;
                const int xm = active ? row % (BW > 1 ? BW : M2) : 0;
                int lrow[NW];
                bool row_ok[NW];
                lrow[0] = (ly + dy) * pitch + (lx + xm);
                row_ok[0] = active;
                if constexpr (NW > 1) {
                    lrow[1] = lrow[0] + BW;
                    row_ok[1] = xm < BW - 1;  // column lx + 15 is outside every footprint
                }
                const int qshift = U - g.z0 - M2;  // slab-relative plane = q + qshift

                R wr[NW][M2], wi[NW][M2];
#pragma unroll
                for (int w = 0; w < NW; ++w)
#pragma unroll
                    for (int s = 0; s < M2; ++s) wr[w][s] = wi[w][s] = R(0);

                // add slot s (plane q) of the lane's rows into the LDS tile
                auto flush = [&](int s, int q) __attribute__((always_inline)) {
                    const int o = (q + qshift) * plane;
                    if constexpr (COMP) {
                        unsigned long long *c[2 * NW];
                        float v[2 * NW];
                        bool ok[2 * NW];
#pragma unroll
                        for (int w = 0; w < NW; ++w) {
                            c[2 * w] = row_ok[w] ? &pairs[o + lrow[w]] : still;
                            c[2 * w + 1] = row_ok[w] ? &pairs[o + lrow[w] + im_off] : still;
                            v[2 * w] = (float)wr[w][s];
                            v[2 * w + 1] = (float)wi[w][s];
                            ok[2 * w] = ok[2 * w + 1] = row_ok[w];
                        }
                        lds_add_comp<2 * NW>(c, v, ok);
                    } else {
#pragma unroll
                        for (int w = 0; w < NW; ++w) {
                            if (row_ok[w]) {
                                atomicAdd(&acc[o + lrow[w]], wr[w][s]);
                                atomicAdd(&acc[o + lrow[w] + im_off], wi[w][s]);
                            }
                        }
                    }
                };

                // Plane-major sweep: plane q (in window units, q = first
                // tap plane + 2m) lives in slot q mod 2m.  The plane loop is
                // unrolled 2m times, so the slot to retire is a constant;
                // points whose window starts at plane p are added before p
                // is retired (after that, their slot is reused for p + 2m).
                // Only planes f_lo .. f_lo + nf - 1 lie in the slab; the
                // others are dropped.
                const int2 h0 = head_of(stage, a, ST16, OFF_PZ);
                const int B0 = uni(h0.x) + m + 1;
                const int Blast = plane_of(stage, b - 1, ST16, OFF_PZ, m);
                int jn = uni(h0.y);
                const int f_lo = max(B0, -qshift);
                const int nf = max(min(Blast + M2 - 1, g.zs - 1 - qshift) - f_lo + 1, 0);
                const int p_end = max(Blast, f_lo + nf - 1);
                int sl = a, Bn = B0, last = B0;
                int p = B0 - B0 % M2;
                while (p <= p_end) {
#pragma unroll
                    for (int k = 0; k < M2; ++k) {
                        while (Bn == p) {
                            const R *ps = reinterpret_cast<const R *>(stage + sl * ST16);
                            // the next point's header loads while this one is added
                            const int2 hx = head_of(stage, min(sl + 1, b - 1), ST16, OFF_PZ);
                            R sr[NW], si[NW];
                            if constexpr (NW > 1) {
                                // the record holds dim 2 in lane order (slot xm =
                                // tap (xm - j) mod 2m), so the lane reads slot xm
                                const bool hi = xm < jn;
                                const R w12 = ps[M2 + dy] * ps[2 * M2 + xm];
                                const R fr = ps[OFF_F] * w12, fi = ps[OFF_F + 1] * w12;
                                sr[0] = hi ? R(0) : fr;
                                si[0] = hi ? R(0) : fi;
                                sr[1] = hi ? fr : R(0);
                                si[1] = hi ? fi : R(0);
                            } else {
                                const R w12 = active ? ps[M2 + dy] * ps[2 * M2 + xm] : R(0);
                                sr[0] = ps[OFF_F] * w12;
                                si[0] = ps[OFF_F + 1] * w12;
                            }
#pragma unroll
                            for (int s = 0; s < M2; ++s) {
                                const R wz = ps[s];
#pragma unroll
                                for (int w = 0; w < NW; ++w) {
                                    wr[w][s] = fma(sr[w], wz, wr[w][s]);
                                    wi[w][s] = fma(si[w], wz, wi[w][s]);
                                }
                            }
                            last = p;
                            ++sl;
                            Bn = sl < b ? uni(hx.x) + m + 1 : kNoPlane;
                            jn = uni(hx.y);
                        }
                        if ((unsigned)(p - f_lo) < (unsigned)nf) flush(k, p);
#pragma unroll
                        for (int w = 0; w < NW; ++w) wr[w][k] = wi[w][k] = R(0);
                        ++p;
                    }
                    // window empty and the next point far ahead: skip the gap
                    if (last + M2 <= p && Bn != kNoPlane && Bn - Bn % M2 > p) p = Bn - Bn % M2;
                }
              }
            }
            __syncthreads();
            if (more) {
                chunk_store<PF, R>(cntn, slot_n, ST16, rec, rs16, vs, reg, stage);
                __syncthreads();
            }
        }

        const gptr<R> grid = as_global(reinterpret_cast<R *>(xfs[items[it].xf].grid));
        for (int i = tid; i < nz; i += nthr) {
            int z = i / (g.nrows * P), rem = i - z * g.nrows * P;
            int y = g.ry0 + rem / P, xx = rem % P;
            const int o = z * plane + y * pitch + xx;
            R vr, vi;
            if (COMP) {
                unsigned long long a0 = pairs[o], a1 = pairs[o + im_off];
                vr = (R)(__uint_as_float((unsigned int)a0) + __uint_as_float((unsigned int)(a0 >> 32)));
                vi = (R)(__uint_as_float((unsigned int)a1) + __uint_as_float((unsigned int)(a1 >> 32)));
            } else {
                vr = acc[o];
                vi = acc[o + im_off];
            }
            int gy = wrapn(g.Y0 + y - m + 1, g.n1), gx = wrapn(g.X0 + xx - m + 1, g.n2);
            size_t gi = (((size_t)(g.z0 + z) * g.n1 + gy) * g.n2 + gx) * 2;
            if (vr != R(0)) __hip_atomic_fetch_add(&grid[gi], vr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (vi != R(0)) __hip_atomic_fetch_add(&grid[gi + 1], vi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    release_queue(queue);
}

// ---------------------------------------------------------------------------
// Interpolation.  Output per sorted point (atomically added to `outs`, which
// the caller zeroes): one complex value, or with GRAD four complex values
// (value, d/dx0, d/dx1, d/dx2).
template <typename R, int M2, bool GRAD>
__global__ __launch_bounds__(interp_max_threads(sizeof(R), M2, GRAD)) void k_interp(
    const Xform *__restrict__ xfs, const SItem *__restrict__ items, int nitems, int *__restrict__ queue,
    int T, int Zs, int cap, const v4u *__restrict__ rec, int rs16, const int *__restrict__ cell_start,
    R *__restrict__ outs)
{
    constexpr int m = M2 / 2;
    constexpr int ROWS = M2 * M2;
    constexpr int NRG = (ROWS + 63) / 64;
    constexpr int NO = GRAD ? 4 : 1;
    const ValueSlot vs{nullptr, 0, 0};  // interpolation does not read the values
    constexpr int ST16 = (int)(rec_size(M2, sizeof(R), GRAD) / 16);
    constexpr int OFF_PZ = (int)(rec_off_pz(M2, sizeof(R)) / 4);
    constexpr int OFF_D = (int)(rec_prefix(M2, sizeof(R)) / sizeof(R));
    static_assert(rec_off_xr(M2, sizeof(R)) == rec_off_pz(M2, sizeof(R)) + 4 && rec_off_pz(M2, sizeof(R)) % 8 == 0,
                  "head_of reads the plane index and line offset as one int2");
    constexpr int BW = block_w(M2);
    constexpr int NW = BW > 1 ? 2 : 1;  // tile rows per lane
    extern __shared__ uint4 smem16[];
    unsigned char *smem = reinterpret_cast<unsigned char *>(smem16);
    __shared__ int s_item;
    const LdsLayout LL = lds_layout(T, Zs, M2, sizeof(R), GRAD ? 2 : 1, false, cap);
    const int LPR = T / BW;  // runs (blocks of lines) per tile row
    const int P = T + M2 - 1;
    const int plane = P * P;
    R *tile = reinterpret_cast<R *>(smem + LL.tile);
    v4u *stage = reinterpret_cast<v4u *>(smem + LL.stage);
    int *slot_a = reinterpret_cast<int *>(smem + LL.slot_p);
    int *slot_b = slot_a + cap;
    int *run_p0 = reinterpret_cast<int *>(smem + LL.run_p0);
    int *run_soff = reinterpret_cast<int *>(smem + LL.run_soff);
    int *sh = reinterpret_cast<int *>(smem + LL.sh);
    R *oacc = reinterpret_cast<R *>(smem + LL.out);
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int wave = uni(tid >> 6), lane = tid & 63, nwaves = nthr >> 6;
    constexpr int PF = (sizeof(R) == 8 && M2 >= 12) || GRAD ? 2 : 4;

    for (int it = next_item(queue, &s_item); it < nitems; it = next_item(queue, &s_item)) {
        const ItemGeom g = item_geom(items[it], xfs[items[it].xf], T, Zs, M2);
        const int nz = g.zs * g.nrows * P;
        const gptr<const R> grid = as_global(reinterpret_cast<const R *>(xfs[items[it].xf].grid));
        for (int i = tid; i < nz; i += nthr) {
            int z = i / (g.nrows * P), rem = i - z * g.nrows * P;
            int y = g.ry0 + rem / P, xx = rem % P;
            int gy = wrapn(g.Y0 + y - m + 1, g.n1), gx = wrapn(g.X0 + xx - m + 1, g.n2);
            size_t gi = (((size_t)(g.z0 + z) * g.n1 + gy) * g.n2 + gx) * 2;
            const int o = (z * plane + y * P + xx) * 2;
            tile[o] = grid[gi];
            tile[o + 1] = grid[gi + 1];
        }
        const int nr = 3 * (g.le - g.lb);
        const int S = build_runs<M2>(g, T, cell_start, run_p0, run_soff, sh);

        const int nch = (S + cap - 1) / cap;
        v4u reg[PF];
        if (nch > 0) {
            const int c0n = min(cap, S);
            chunk_slots(0, c0n, nr, run_p0, run_soff, slot_a);
            __syncthreads();
            chunk_fetch<PF, R>(c0n, slot_a, ST16, rec, rs16, vs, reg);
            chunk_store<PF, R>(c0n, slot_a, ST16, rec, rs16, vs, reg, stage);
            __syncthreads();
        }
        for (int ch = 0; ch < nch; ++ch) {
            const int cs = ch * cap;
            const int cnt = min(cap, S - cs);
            int *slot_p = (ch & 1) ? slot_b : slot_a;
            int *slot_n = (ch & 1) ? slot_a : slot_b;
            const bool more = ch + 1 < nch;
            const int cntn = more ? min(cap, S - cs - cap) : 0;
            if (more) {
                chunk_slots(cs + cap, cntn, nr, run_p0, run_soff, slot_n);
                __syncthreads();
                chunk_fetch<PF, R>(cntn, slot_n, ST16, rec, rs16, vs, reg);
            }
            // Tasks as in the spread (ranges for blocks of lines, one run for
            // single lines); a task evaluates each run piece it covers (all
            // row groups), 64 points at a time, one lane owning the outputs
            // of each point, so every slot has exactly one writer.
            const int r_lo = uni(find_run(run_soff, nr, cs));
            const int r_hi = uni(find_run(run_soff, nr, cs + cnt - 1));
            const int piece = max(16, (cnt + nwaves - 1) / nwaves);
            const int ntask = BW > 1 ? (cnt + piece - 1) / piece : r_hi - r_lo + 1;
            for (int task = wave; task < ntask; task += nwaves) {
              int lo = cs, hi = cs + cnt, rf = r_lo + task;
              if (BW > 1) {
                  lo = cs + task * piece;
                  hi = min(cs + cnt, lo + piece);
                  rf = uni(find_run(run_soff, nr, lo));
              }
              for (int r = rf; r < nr && uni(run_soff[r]) < hi && (BW > 1 || r == rf); ++r) {
                const int a = uni(max(run_soff[r], lo) - cs);
                const int b = uni(min(run_soff[r + 1], hi) - cs);
                if (a >= b) continue;
                const int li = g.lb + r / 3;
                const int U = (r % 3 - 1) * g.n0;
                const int ly = li / LPR, lx = (li % LPR) * BW;  // the run's first line
                const int qshift = U - g.z0 - M2;
                for (int c0 = a; c0 < b; c0 += 64) {
                    const int c1 = min(b, c0 + 64);
                    R ores[2 * NO];
#pragma unroll
                    for (int i = 0; i < 2 * NO; ++i) ores[i] = R(0);
                    for (int rg = 0; rg < NRG; ++rg) {
                        const int row = rg * 64 + lane;
                        const bool active = ROWS % 64 == 0 || row < ROWS;
                        // tile rows of this lane (as in the spread)
                        const int dy = active ? row / (BW > 1 ? BW : M2) : 0;
                        const int xm = active ? row % (BW > 1 ? BW : M2) : 0;
                        int lrow[NW];
                        bool row_ok[NW];
                        lrow[0] = (ly + dy) * P + (lx + xm);
                        row_ok[0] = active;
                        if constexpr (NW > 1) {
                            lrow[1] = lrow[0] + BW;
                            row_ok[1] = xm < BW - 1;
                        }

                        R gr[NW][M2], gi[NW][M2];
#pragma unroll
                        for (int w = 0; w < NW; ++w)
#pragma unroll
                            for (int s = 0; s < M2; ++s) gr[w][s] = gi[w][s] = R(0);
                        // Plane-major sweep (as in the spread): slot q mod 2m
                        // holds plane q; at plane p the plane p + 2m - 1
                        // enters, then the points whose window starts at p
                        // are evaluated.  Partials of consecutive points feed
                        // a binary counter of cross-lane halving steps: level
                        // 1 pairs points, level 2 quads, level 3 octets.
                        auto load = [&](int s, int q) __attribute__((always_inline)) {
                            const int qr = q + qshift;
#pragma unroll
                            for (int w = 0; w < NW; ++w) {
                                if (row_ok[w] && (unsigned)qr < (unsigned)g.zs) {
                                    const int o = (qr * plane + lrow[w]) * 2;
                                    gr[w][s] = tile[o];
                                    gi[w][s] = tile[o + 1];
                                } else {
                                    gr[w][s] = R(0);
                                    gi[w][s] = R(0);
                                }
                            }
                        };
                        R s0[2 * NO], s1[2 * NO], s2[2 * NO];
                        auto feed = [&](int t, R (&v)[2 * NO]) {
                            if (!(t & 1)) {
#pragma unroll
                                for (int i = 0; i < 2 * NO; ++i) s0[i] = v[i];
                                return;
                            }
#pragma unroll
                            for (int i = 0; i < 2 * NO; ++i) v[i] = halve32(s0[i], v[i]);
                            if (!(t & 2)) {
#pragma unroll
                                for (int i = 0; i < 2 * NO; ++i) s1[i] = v[i];
                                return;
                            }
#pragma unroll
                            for (int i = 0; i < 2 * NO; ++i) v[i] = halve16(s1[i], v[i]);
                            if (!(t & 4)) {
#pragma unroll
                                for (int i = 0; i < 2 * NO; ++i) s2[i] = v[i];
                                return;
                            }
                            // octet t-7 .. t complete: 8-lane group j holds
                            // point t - 7 + bitrev3(j); lane 8j + (t >> 3) keeps it
#pragma unroll
                            for (int i = 0; i < 2 * NO; ++i) {
                                const R tot = halve8_sum(s2[i], v[i]);
                                if ((lane & 7) == (t >> 3)) ores[i] += tot;
                            }
                        };
                        int sl = c0;
                        const int2 h0 = head_of(stage, c0, ST16, OFF_PZ);
                        int Bn = uni(h0.x) + m + 1;
                        int jn = uni(h0.y);
                        int p = Bn - Bn % M2;
#pragma unroll
                        for (int s = 0; s < M2 - 1; ++s)
                            if (p + s >= Bn) load(s, p + s);
                        while (sl < c1) {
#pragma unroll
                            for (int k = 0; k < M2; ++k) {
                                if (Bn <= p + M2 - 1) load((k + M2 - 1) % M2, p + M2 - 1);
                                while (Bn == p) {
                                    const R *ps = reinterpret_cast<const R *>(stage + sl * ST16);
                                    const int2 hx = head_of(stage, min(sl + 1, c1 - 1), ST16, OFF_PZ);
                                    // the lane's row for this point: single
                                    // lines use row 0; in a block, row 1 when
                                    // the point's line lies right of column xm
                                    // (dim 2 is stored in lane order: the
                                    // lane's tap is slot xm)
                                    const bool hi = NW > 1 && xm < jn;
                                    R sr, si;
                                    {
                                        R ar[NW], ai[NW];
#pragma unroll
                                        for (int w = 0; w < NW; ++w) {
                                            ar[w] = ai[w] = R(0);
#pragma unroll
                                            for (int s = 0; s < M2; ++s) {
                                                ar[w] = fma(gr[w][s], ps[s], ar[w]);
                                                ai[w] = fma(gi[w][s], ps[s], ai[w]);
                                            }
                                        }
                                        sr = (NW > 1 && hi) ? ar[NW - 1] : ar[0];
                                        si = (NW > 1 && hi) ? ai[NW - 1] : ai[0];
                                    }
                                    const R w1 = active ? ps[M2 + dy] : R(0);
                                    const R w2 = active ? ps[2 * M2 + xm] : R(0);
                                    const R w12 = w1 * w2;
                                    R v[2 * NO];
                                    v[0] = sr * w12;
                                    v[1] = si * w12;
                                    if constexpr (GRAD) {
                                        const R *dp = ps + OFF_D;
                                        R dr, di;
                                        {
                                            R ar[NW], ai[NW];
#pragma unroll
                                            for (int w = 0; w < NW; ++w) {
                                                ar[w] = ai[w] = R(0);
#pragma unroll
                                                for (int s = 0; s < M2; ++s) {
                                                    ar[w] = fma(gr[w][s], dp[s], ar[w]);
                                                    ai[w] = fma(gi[w][s], dp[s], ai[w]);
                                                }
                                            }
                                            dr = (NW > 1 && hi) ? ar[NW - 1] : ar[0];
                                            di = (NW > 1 && hi) ? ai[NW - 1] : ai[0];
                                        }
                                        const R d1 = active ? dp[M2 + dy] * w2 : R(0);
                                        const R d2 = active ? w1 * dp[2 * M2 + xm] : R(0);
                                        v[2] = dr * w12;
                                        v[3] = di * w12;
                                        v[4] = sr * d1;
                                        v[5] = si * d1;
                                        v[6] = sr * d2;
                                        v[7] = si * d2;
                                    }
                                    feed(sl - c0, v);
                                    ++sl;
                                    Bn = sl < c1 ? uni(hx.x) + m + 1 : kNoPlane;
                                    jn = uni(hx.y);
                                }
                                ++p;
                            }
                            // skip a gap: restart the window at the next point
                            if (sl < c1 && Bn - Bn % M2 > p) {
                                p = Bn - Bn % M2;
#pragma unroll
                                for (int s = 0; s < M2 - 1; ++s)
                                    if (p + s >= Bn) load(s, p + s);
                            }
                        }
                        // pad the last octet with zero partials
                        for (int t = c1 - c0; t & 7; ++t) {
                            R v[2 * NO];
#pragma unroll
                            for (int i = 0; i < 2 * NO; ++i) v[i] = R(0);
                            feed(t, v);
                        }
                    }
                    const int j8 = lane >> 3;
                    const int own = (lane & 7) * 8 + (((j8 & 1) << 2) | (j8 & 2) | (j8 >> 2));
                    if (own < c1 - c0) {
#pragma unroll
                        for (int i = 0; i < 2 * NO; ++i) oacc[(c0 + own) * 2 * NO + i] = ores[i];
                    }
                }
              }
            }
            __syncthreads();
            for (int e = tid; e < cnt * 2 * NO; e += nthr) {
                R v = oacc[e];
                if (v != R(0)) atomicAdd(&outs[(size_t)slot_p[e / (2 * NO)] * (2 * NO) + e % (2 * NO)], v);
            }
            __syncthreads();
            if (more) {
                chunk_store<PF, R>(cntn, slot_n, ST16, rec, rs16, vs, reg, stage);
                __syncthreads();
            }
        }
    }
    release_queue(queue);
}

// ---------------------------------------------------------------------------
static int cu_count()
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

// Two workgroups per compute unit, each with half the LDS and at most 512
// threads, when the tile leaves both a staging area worth having: kTwoWgCap
// points, or fewer when the work items hold fewer (cap_hint, from the
// binning).  One workgroup's list, staging and flush phases (barriers and
// HBM latency) then overlap the other's sweep.
constexpr int kTwoWgCap = 256;
static void two_per_cu(LdsLayout &LL, const Tiling &t, int M2, size_t R, int kind, bool comp, int &threads)
{
    int need = kTwoWgCap;
    if (t.cap_hint > 0) need = std::min(need, std::max(64, t.cap_hint));
    int cap = LL.cap;
    while (cap >= need && 2 * (lds_layout(t.T, t.Zs, M2, R, kind, comp, cap).total + 1024) > 160 * 1024) cap -= 16;
    if (cap < need || cap < 16) return;
    LL = lds_layout(t.T, t.Zs, M2, R, kind, comp, cap);
    threads = std::max(64, std::min(threads, 512));
}

template <typename R, int M2>
static hipError_t spread_m(const Xform *dxf, const SItem *items, int nitems, int *queue, Tiling t,
                           const unsigned char *rec, size_t rec_bytes, const R *fs, const int *cs, hipStream_t s)
{
    constexpr bool COMP = sizeof(R) == 4;
    LdsLayout LL = lds_fit(t.T, t.Zs, M2, sizeof(R), 0, COMP);
    if (!LL.cap) return hipErrorInvalidValue;
    int threads = std::min(t.threads, spread_max_threads(sizeof(R), M2));
    two_per_cu(LL, t, M2, sizeof(R), 0, COMP, threads);
    auto kern = k_spread<R, M2, COMP>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)LL.total);
    if (e != hipSuccess) return e;
    int per_cu = (int)((160 * 1024) / (LL.total + 1024));
    if (per_cu < 1) per_cu = 1;
    int grid = std::min(cu_count() * per_cu, nitems);
    if (grid < 1) return hipSuccess;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(threads), LL.total, s, dxf, items, nitems, queue, t.T, t.Zs,
                       LL.cap, (const v4u *)rec, (int)(rec_bytes / 16), fs, cs);
    return hipGetLastError();
}

template <typename R, int M2, bool GRAD>
static hipError_t interp_m(const Xform *dxf, const SItem *items, int nitems, int *queue, Tiling t,
                           const unsigned char *rec, size_t rec_bytes, const int *cs, R *outs, hipStream_t s)
{
    LdsLayout LL = lds_fit(t.T, t.Zs, M2, sizeof(R), GRAD ? 2 : 1, false);
    if (!LL.cap) return hipErrorInvalidValue;
    int threads = std::min(t.threads, interp_max_threads(sizeof(R), M2, GRAD));
    two_per_cu(LL, t, M2, sizeof(R), GRAD ? 2 : 1, false, threads);
    auto kern = k_interp<R, M2, GRAD>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)LL.total);
    if (e != hipSuccess) return e;
    int per_cu = (int)((160 * 1024) / (LL.total + 1024));
    if (per_cu < 1) per_cu = 1;
    int grid = std::min(cu_count() * per_cu, nitems);
    if (grid < 1) return hipSuccess;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(threads), LL.total, s, dxf, items, nitems, queue, t.T, t.Zs,
                       LL.cap, (const v4u *)rec, (int)(rec_bytes / 16), cs, outs);
    return hipGetLastError();
}

}  // namespace hpnfft
