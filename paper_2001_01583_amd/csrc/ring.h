// Ring sweeps for windows of 2m = 8 cells, on the blocked-line layout of
// sweep.h: the spread (the Spreading step of Algorithm 2, Section 3) here,
// the interpolation (the Interpolating step of Algorithm 5) below.
//
// A work item is a tile of 8 x 8 z-lines (eight blocks of 8 lines, one per
// tile row) restricted to a slab of Zs planes along dim 0.  Each wavefront
// owns one block and sweeps, in plane order, the block's points whose
// windows reach the slab (the periodic images of the line segment come in
// plane order by themselves), retiring the slab's planes only.  (Sweeping
// each point once, in the slab of its first tap plane, and retiring the
// 2m - 1 planes past the slab as well, measured slower: 0.233 against 0.215
// ms at N = 64^3, M = 2^20, float32, 32-plane slabs.)  The per-point values
// that are the same on every lane (dim-0 weights, the value, the header)
// come through scalar loads; the lane's own dim-1 and dim-2 weights are one
// load each from fixed slots of the record (dim 2 is stored in lane order).
//
// The blocks of one tile overlap in their tap rows, so their retired planes
// meet in LDS: a ring of kRingZp = 2m planes, one phase.  In phase k the
// wavefronts retire planes [k Zp, (k + 1) Zp); after a barrier all threads
// add the ring to the grid (one atomic per cell) and clear it, and a second
// barrier opens the next phase.  Register windows (the planes still open
// when a phase ends) carry over to the next phase.  The ring is small (30
// KiB) so that four workgroups share a compute unit and hide each other's
// barriers and load latencies.
#pragma once

#include "sweep.h"

namespace hpnfft {

constexpr int kRingP = kRingT + 7;  // footprint rows (and used columns) of a tile
constexpr int kRingPitch = 16;   // cells per LDS row; column 15 only ever receives zeros
constexpr int kRingPlane = kRingP * kRingPitch;
constexpr int kRingThreads = 512;  // eight wavefronts: one per block of the tile
constexpr size_t kRingLds = (size_t)kRingZp * kRingPlane * 16;  // re and im arrays of 8-byte cells

// Wavefronts per SIMD the register budget is set for: the ring takes 30 KiB
// of LDS, so four workgroups (eight wavefronts per SIMD, 64 registers per
// lane) fit in float32; the float64 sweep holds twice the window in
// registers and keeps four wavefronts per SIMD.
template <typename R> constexpr int ring_waves_per_simd() { return sizeof(R) == 4 ? 8 : 4; }

template <typename R, bool COMP>
__global__ __launch_bounds__(kRingThreads, ring_waves_per_simd<R>()) void k_spread_ring(const Xform *__restrict__ xfs,
                                                               const SItem *__restrict__ items, int nitems,
                                                               int *__restrict__ queue, int Zs,
                                                               const unsigned char *__restrict__ rec, int rbytes,
                                                               const R *__restrict__ fs,
                                                               const int *__restrict__ cell_start)
{
    constexpr int M2 = 8, m = 4, BW = 8;
    constexpr int NRP = kRingZp;           // ring planes
    constexpr int IM = NRP * kRingPlane;   // cells before the imaginary array
    constexpr int OFF_PZ = (int)rec_off_pz(M2, sizeof(R));
    static_assert((NRP & (NRP - 1)) == 0, "ring planes: a power of two");
    extern __shared__ uint4 smem16[];
    unsigned long long *pairs = reinterpret_cast<unsigned long long *>(smem16);
    R *acc = reinterpret_cast<R *>(smem16);
    __shared__ int s_item;
    const int tid = threadIdx.x, lane = tid & 63, wave = uni(tid >> 6);
    const int dy = lane >> 3, xm = lane & 7;

    // the flushes leave every cell they read at zero
    for (int i = tid; i < 2 * IM; i += blockDim.x) pairs[i] = 0ull;

    for (int it = next_item(queue, &s_item); it < nitems; it = next_item(queue, &s_item)) {
        const SItem W = items[uni(it)];
        const Xform *X = xfs + W.xf;
        const int n0 = X->n[0], n1 = X->n[1], n2 = X->n[2];
        const int ntx = X->ntx;
        const int X0 = (W.tile % ntx) * kRingT, Y0 = (W.tile / ntx) * kRingT;
        const int z0 = W.slab * Zs, zs = min(Zs, n0 - z0);
        const long long poff = X->poff;
        const int li = W.lb + wave;  // this wavefront's block (tile row li)
        const bool mine = li < W.le && Y0 + li < n1;

        // The block's points by plane: sorted positions [cs[8 c], cs[8 (c + 1)])
        // hold plane c of the block (every line).  Slab-relative plane q is
        // the first tap plane of the points in grid plane c = q + m - 1 + z0
        // (mod n0): the periodic images of the line segment come in plane
        // order by themselves.
        const int *cs = cell_start + X->key_off + ((long long)W.tile * (kRingT * kRingT / BW) + li) * n0 * BW;
        const int Mx = (int)X->M;
        auto plane_c = [&](int q) __attribute__((always_inline)) {
            int c = q + (m - 1) + z0;  // within [-m, 2 n0)
            c += c < 0 ? n0 : 0;
            c -= c >= n0 ? n0 : 0;
            return c;
        };

        // Point data, one point ahead: the loads of the next point in memory
        // are in flight while the current one is added (a point whose data
        // was not prefetched, the first of a plane after a periodic wrap, is
        // loaded when it is reached).
        struct PointData {
            R wz[M2];
            R f0, f1, wy, wx;
            int j;
        };
        // (the wavefront-uniform parts are read as constant memory, i.e.
        // through scalar loads: records and values do not change while the
        // kernel runs)
        const unsigned char *recb = rec + (size_t)poff * rbytes;
        const R *fsb = fs + 2 * poff;
        auto fetch = [&](const unsigned char *rp, const R *fp, PointData &d) __attribute__((always_inline)) {
            const cptr<R> pc = as_const(reinterpret_cast<const R *>(rp));
#pragma unroll
            for (int s = 0; s < M2; ++s) d.wz[s] = pc[s];
            d.j = as_const(reinterpret_cast<const int *>(rp + OFF_PZ))[1];
            d.f0 = as_const(fp)[0];
            d.f1 = as_const(fp)[1];
            const R *ps = reinterpret_cast<const R *>(rp);
            d.wy = ps[M2 + dy];
            d.wx = ps[2 * M2 + xm];
        };
        PointData cur{};
        int cidx = -1;  // point whose data cur holds
        const unsigned char *rcur = recb;  // its record
        const R *fcur = fsb;               // its value

        R wr[2][M2], wi[2][M2];
#pragma unroll
        for (int w = 0; w < 2; ++w)
#pragma unroll
            for (int s = 0; s < M2; ++s) wr[w][s] = wi[w][s] = R(0);

        const int rowc = (li + dy) * kRingPitch + xm;  // lane's first cell in a ring plane
        int last = -1000;  // first tap plane of the last point added
        // sorted range of the next plane to sweep, loaded one plane ahead
        // (the first plane with points is -(2m - 1): windows that end on
        // the slab's first plane)
        int na = 0, nb = 0;
        if (mine) {
            const int c = plane_c(-(M2 - 1));
            na = cs[c * BW];
            nb = cs[(c + 1) * BW];
        }

        // plane q: add its points, retire slot k = q mod 2m (if in this
        // phase's planes and reached by some window), clear the slot
        auto plane_step = [&](const int k, const int q, const int pe) __attribute__((always_inline)) {
            if (q >= -(M2 - 1) && q < zs) {
                const int pa = uni(na), pb = uni(nb);
                const int c = plane_c(q + 1);
                na = cs[c * BW];
                nb = cs[(c + 1) * BW];
                for (int sp = pa; sp < pb; ++sp) {
                    if (sp != cidx) {
                        rcur = recb + (size_t)sp * rbytes;
                        fcur = fsb + 2 * sp;
                        fetch(rcur, fcur, cur);
                    }
                    const bool adv = sp + 1 < Mx;
                    const unsigned char *rnx = adv ? rcur + rbytes : rcur;
                    const R *fnx = adv ? fcur + 2 : fcur;
                    PointData nxt;
                    fetch(rnx, fnx, nxt);
                    const int j = uni(cur.j);
                    const R w12 = cur.wy * cur.wx;
                    const R fr = cur.f0 * w12, fi = cur.f1 * w12;
                    // a point on line j reaches column xm (tap xm - j) when
                    // xm >= j, else column xm + 8
                    const bool hi = xm < j;
                    const R s0r = hi ? R(0) : fr, s0i = hi ? R(0) : fi;
                    const R s1r = hi ? fr : R(0), s1i = hi ? fi : R(0);
#pragma unroll
                    for (int s = 0; s < M2; ++s) {
                        const R wz = cur.wz[s];
                        wr[0][s] = fma(s0r, wz, wr[0][s]);
                        wi[0][s] = fma(s0i, wz, wi[0][s]);
                        wr[1][s] = fma(s1r, wz, wr[1][s]);
                        wi[1][s] = fma(s1i, wz, wi[1][s]);
                    }
                    cur = nxt;
                    cidx = adv ? sp + 1 : sp;
                    rcur = rnx;
                    fcur = fnx;
                }
                if (pb > pa) last = q;
            }
            if (q >= 0 && q < pe && last + M2 > q) {
                const int o = (q & (NRP - 1)) * kRingPlane + rowc;
                if constexpr (COMP) {
                    unsigned long long *c[4] = {&pairs[o], &pairs[o + 8], &pairs[o + IM], &pairs[o + IM + 8]};
                    const float v[4] = {(float)wr[0][k], (float)wr[1][k], (float)wi[0][k], (float)wi[1][k]};
                    const bool ok[4] = {true, true, true, true};
                    lds_add_comp<4>(c, v, ok);
                } else {
                    atomicAdd(&acc[o], wr[0][k]);
                    atomicAdd(&acc[o + IM], wi[0][k]);
                    if (xm < 7) {
                        atomicAdd(&acc[o + 8], wr[1][k]);
                        atomicAdd(&acc[o + IM + 8], wi[1][k]);
                    }
                }
            }
            wr[0][k] = wi[0][k] = wr[1][k] = wi[1][k] = R(0);
        };

        // planes in groups of 2m (slot k of plane p + k, p a multiple of 2m);
        // a phase is one group
        int p = -M2;
        const int nph = (zs + kRingZp - 1) / kRingZp;
        for (int ph = 0; ph < nph; ++ph) {
            const int pe = min((ph + 1) * kRingZp, zs);  // planes below pe retire in this phase
            if (mine) {
                for (; p < pe; p += M2) {
#pragma unroll
                    for (int k = 0; k < M2; ++k) plane_step(k, p + k, pe);
                }
            }
            __syncthreads();
            // add this phase's planes to the grid and clear them
            const int zb = ph * kRingZp, nzp = pe - zb;
            const int ry0 = W.lb, ry1 = min(W.le, n1 - Y0) + M2 - 1;  // rows any block reached
            const size_t pstride = (size_t)n1 * n2;
            const gptr<R> grid = as_global(reinterpret_cast<R *>(X->grid));
            for (int i = tid; i < nzp * kRingPlane; i += blockDim.x) {
                const int zz = i / kRingPlane, c = i - zz * kRingPlane;
                const int y = c / kRingPitch, x = c % kRingPitch;
                if (y < ry0 || y >= ry1 || x >= kRingP) continue;
                const int o = ((zb + zz) & (NRP - 1)) * kRingPlane + c;
                R vr, vi;
                if constexpr (COMP) {
                    const unsigned long long a0 = pairs[o], a1 = pairs[o + IM];
                    vr = (R)(__uint_as_float((unsigned int)a0) + __uint_as_float((unsigned int)(a0 >> 32)));
                    vi = (R)(__uint_as_float((unsigned int)a1) + __uint_as_float((unsigned int)(a1 >> 32)));
                } else {
                    vr = acc[o];
                    vi = acc[o + IM];
                }
                pairs[o] = 0ull;
                pairs[o + IM] = 0ull;
                int gy = Y0 + y - (m - 1), gx = X0 + x - (m - 1);
                gy += gy < 0 ? n1 : 0;
                gy -= gy >= n1 ? n1 : 0;
                gy -= gy >= n1 ? n1 : 0;
                gx += gx < 0 ? n2 : 0;
                gx -= gx >= n2 ? n2 : 0;
                gx -= gx >= n2 ? n2 : 0;
                const size_t gi = ((size_t)(z0 + zb + zz) * pstride + (size_t)gy * n2 + gx) * 2;
                if (vr != R(0)) __hip_atomic_fetch_add(&grid[gi], vr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (vi != R(0)) __hip_atomic_fetch_add(&grid[gi + 1], vi, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            // the next phase retires into the same planes
            if (ph + 1 < nph) __syncthreads();
        }
    }
    release_queue(queue);
}

// Interpolation (the Interpolating step of Algorithm 5) for 2m = 8 on the
// same items.  A point is evaluated by the slab that holds its first tap
// plane, in full: the ring carries the slab's planes and the 2m - 1 planes
// past its end.  Per phase all threads copy the next 2m planes of the tile
// footprint from the grid into the LDS ring; each wavefront then takes one
// step per plane q: plane q enters register slot q mod 2m of the lane's two
// columns, and the block's points whose window starts at q - 2m + 1 (now
// complete in registers) are evaluated.  The per-lane partials of
// consecutive points go through the halving steps of wave_reduce.h; every
// 64 points each lane holds one point's sum and stores it (every point has
// exactly one writer, so the output needs neither atomics nor clearing).
template <typename R>
__global__ __launch_bounds__(kRingThreads, ring_waves_per_simd<R>()) void k_interp_ring(
    const Xform *__restrict__ xfs, const SItem *__restrict__ items, int nitems, int *__restrict__ queue, int Zs,
    const unsigned char *__restrict__ rec, int rbytes, const int *__restrict__ cell_start, R *__restrict__ outs)
{
    constexpr int M2 = 8, m = 4, BW = 8;
    constexpr int NRP = kRingZp;
    constexpr int OFF_PZ = (int)rec_off_pz(M2, sizeof(R));
    static_assert(kRingZp == M2, "a phase is one group of 2m planes");
    extern __shared__ uint4 smem16[];
    R *ring = reinterpret_cast<R *>(smem16);  // [plane][row][column] complex
    __shared__ int s_item;
    const int tid = threadIdx.x, lane = tid & 63, wave = uni(tid >> 6);
    const int dy = lane >> 3, xm = lane & 7;
    // batch position whose sum this lane receives (see halve8_sum)
    const int own = (lane & 7) * 8 + (((dy & 1) << 2) | (dy & 2) | (dy >> 2));

    for (int i = tid; i < 2 * NRP * kRingPlane; i += blockDim.x) ring[i] = R(0);

    for (int it = next_item(queue, &s_item); it < nitems; it = next_item(queue, &s_item)) {
        const SItem W = items[uni(it)];
        const Xform *X = xfs + W.xf;
        const int n0 = X->n[0], n1 = X->n[1], n2 = X->n[2];
        const int ntx = X->ntx;
        const int X0 = (W.tile % ntx) * kRingT, Y0 = (W.tile / ntx) * kRingT;
        const int z0 = W.slab * Zs, zs = min(Zs, n0 - z0);
        const long long poff = X->poff;
        const int li = W.lb + wave;
        const bool mine = li < W.le && Y0 + li < n1;
        const int *cs = cell_start + X->key_off + ((long long)W.tile * (kRingT * kRingT / BW) + li) * n0 * BW;
        const int Mx = (int)X->M;
        auto plane_c = [&](int q) __attribute__((always_inline)) {
            int c = q + (m - 1) + z0;
            c += c < 0 ? n0 : 0;
            c -= c >= n0 ? n0 : 0;
            return c;
        };
        struct PointData {
            R wz[M2];
            R wy, wx;
            int j;
        };
        const unsigned char *recb = rec + (size_t)poff * rbytes;
        auto fetch = [&](const unsigned char *rp, PointData &d) __attribute__((always_inline)) {
            const cptr<R> pc = as_const(reinterpret_cast<const R *>(rp));
#pragma unroll
            for (int s = 0; s < M2; ++s) d.wz[s] = pc[s];
            d.j = as_const(reinterpret_cast<const int *>(rp + OFF_PZ))[1];
            const R *ps = reinterpret_cast<const R *>(rp);
            d.wy = ps[M2 + dy];
            d.wx = ps[2 * M2 + xm];
        };
        PointData cur{};
        int cidx = -1;
        // partial sums of the last point evaluated, not yet reduced
        R pvr = 0, pvi = 0;
        int pend = -1;  // its sorted index (-1: none)
        const unsigned char *rcur = recb;

        R gr[2][M2], gi[2][M2];
#pragma unroll
        for (int w = 0; w < 2; ++w)
#pragma unroll
            for (int s = 0; s < M2; ++s) gr[w][s] = gi[w][s] = R(0);

        // halving-step state: partials of the open pair, quad and octet
        R s0r = 0, s0i = 0, s1r = 0, s1i = 0, s2r = 0, s2i = 0, orr = 0, ori = 0;
        int t = 0;       // position of the next point in the batch of 64
        int bsp = 0;     // lane t: sorted index of batch point t
        auto feed = [&](R vr, R vi) __attribute__((always_inline)) {
            if (!(t & 1)) {
                s0r = vr;
                s0i = vi;
            } else {
                vr = halve32(s0r, vr);
                vi = halve32(s0i, vi);
                if (!(t & 2)) {
                    s1r = vr;
                    s1i = vi;
                } else {
                    vr = halve16(s1r, vr);
                    vi = halve16(s1i, vi);
                    if (!(t & 4)) {
                        s2r = vr;
                        s2i = vi;
                    } else {
                        const R tr = halve8_sum(s2r, vr), ti = halve8_sum(s2i, vi);
                        if ((lane & 7) == (t >> 3)) {
                            orr += tr;
                            ori += ti;
                        }
                    }
                }
            }
            ++t;
        };
        // every lane that holds the sum of a point stores it (positions
        // padded with zeros hold no point); then the batch restarts
        auto drain = [&]() __attribute__((always_inline)) {
            const int count = t;
            while (t & 7) feed(R(0), R(0));
            const int sp_own = __builtin_amdgcn_ds_bpermute(own << 2, bsp);
            if (own < count) {
                outs[(size_t)sp_own * 2] = orr;
                outs[(size_t)sp_own * 2 + 1] = ori;
            }
            orr = ori = R(0);
            t = 0;
        };
        auto reduce_pending = [&]() __attribute__((always_inline)) {
            bsp = lane == t ? (int)(poff + pend) : bsp;
            feed(pvr, pvi);
            if (t == 64) drain();
            pend = -1;
        };

        // sorted point range of base plane b (b < zs <= 64) in lane b: read
        // with lane reads at the steps, so that the steps wait on no load
        int rlo = 0, rhi = 0;
        if (mine && lane < zs) {
            const int c = plane_c(lane);
            rlo = cs[c * BW];
            rhi = cs[(c + 1) * BW];
        }
        const int zr = zs + M2 - 1;  // planes the ring carries: the slab and the windows past it
        const int rowc = (li + dy) * kRingPitch + xm;
        // step q: plane q (slot k = q mod 2m) enters from the ring; then the
        // points whose window starts at q - 2m + 1
        auto step = [&](const int k, const int q) __attribute__((always_inline)) {
            if (q < zr) {
                const int o = ((q & (NRP - 1)) * kRingPlane + rowc) * 2;
                gr[0][k] = ring[o];
                gi[0][k] = ring[o + 1];
                gr[1][k] = ring[o + 16];
                gi[1][k] = ring[o + 17];
            } else {
                gr[0][k] = gi[0][k] = gr[1][k] = gi[1][k] = R(0);
            }
            const int b = q - (M2 - 1);
            if (b >= 0 && b < zs) {
                const int pa = __builtin_amdgcn_readlane(rlo, b), pb = __builtin_amdgcn_readlane(rhi, b);
                for (int sp = pa; sp < pb; ++sp) {
                    // the previous point's reduction runs first, so that this
                    // point's loads (issued right after the previous point's
                    // sums, into the same registers) are in flight meanwhile
                    if (pend >= 0) reduce_pending();
                    if (sp != cidx) {
                        rcur = recb + (size_t)sp * rbytes;
                        fetch(rcur, cur);
                    }
                    R a0r = 0, a0i = 0, a1r = 0, a1i = 0;
#pragma unroll
                    for (int s = 0; s < M2; ++s) {
                        const R wz = cur.wz[s];
                        a0r = fma(gr[0][s], wz, a0r);
                        a0i = fma(gi[0][s], wz, a0i);
                        a1r = fma(gr[1][s], wz, a1r);
                        a1i = fma(gi[1][s], wz, a1i);
                    }
                    // the lane's column for a point on line j: xm if xm >= j,
                    // else xm + 8
                    const bool hi = xm < uni(cur.j);
                    const R w12 = cur.wy * cur.wx;
                    pvr = (hi ? a1r : a0r) * w12;
                    pvi = (hi ? a1i : a0i) * w12;
                    pend = sp;
                    const bool adv = sp + 1 < Mx;
                    rcur = adv ? rcur + rbytes : rcur;
                    fetch(rcur, cur);
                    cidx = adv ? sp + 1 : sp;
                }
            }
        };

        const int ry0 = W.lb, ry1 = min(W.le, n1 - Y0) + M2 - 1;
        const size_t pstride = (size_t)n1 * n2;
        const gptr<const R> grid = as_global(reinterpret_cast<const R *>(X->grid));
        const int nph = (zr + kRingZp - 1) / kRingZp;
        for (int ph = 0; ph < nph; ++ph) {
            {
                // the phase's planes of the footprint rows the blocks reach
                const int zb = ph * kRingZp;
                for (int i = tid; i < kRingZp * kRingPlane; i += blockDim.x) {
                    const int zz = i / kRingPlane, c = i - zz * kRingPlane;
                    const int y = c / kRingPitch, x = c % kRingPitch;
                    if (zb + zz >= zr || y < ry0 || y >= ry1 || x >= kRingP) continue;
                    int gz = z0 + zb + zz;  // below 2 n0
                    gz -= gz >= n0 ? n0 : 0;
                    int gy = Y0 + y - (m - 1), gx = X0 + x - (m - 1);
                    gy += gy < 0 ? n1 : 0;
                    gy -= gy >= n1 ? n1 : 0;
                    gy -= gy >= n1 ? n1 : 0;
                    gx += gx < 0 ? n2 : 0;
                    gx -= gx >= n2 ? n2 : 0;
                    gx -= gx >= n2 ? n2 : 0;
                    const size_t gi = ((size_t)gz * pstride + (size_t)gy * n2 + gx) * 2;
                    const int o = (((zb + zz) & (NRP - 1)) * kRingPlane + c) * 2;
                    ring[o] = grid[gi];
                    ring[o + 1] = grid[gi + 1];
                }
                __syncthreads();
            }
            if (mine) {
#pragma unroll
                for (int k = 0; k < M2; ++k) step(k, ph * kRingZp + k);
            }
            if (ph + 1 < nph) __syncthreads();
        }
        if (mine && pend >= 0) reduce_pending();
        if (mine && t > 0) drain();
    }
    release_queue(queue);
}

template <typename R>
static hipError_t spread_ring(const Xform *dxf, const SItem *items, int nitems, int *queue, Tiling t,
                              const unsigned char *rec, size_t rec_bytes, const R *fs, const int *cs, hipStream_t s)
{
    constexpr bool COMP = sizeof(R) == 4;
    auto kern = k_spread_ring<R, COMP>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kRingLds);
    if (e != hipSuccess) return e;
    const int per_cu = std::max(1, (int)((160 * 1024) / (kRingLds + 1024)));
    const int grid = std::min(cu_count() * per_cu, nitems);
    if (grid < 1) return hipSuccess;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kRingThreads), kRingLds, s, dxf, items, nitems, queue, t.Zs, rec,
                       (int)rec_bytes, fs, cs);
    return hipGetLastError();
}

template <typename R>
static hipError_t interp_ring(const Xform *dxf, const SItem *items, int nitems, int *queue, Tiling t,
                              const unsigned char *rec, size_t rec_bytes, const int *cs, R *outs, hipStream_t s)
{
    constexpr size_t lds = (size_t)kRingZp * kRingPlane * 2 * sizeof(R);
    auto kern = k_interp_ring<R>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const int per_cu = std::max(1, std::min(ring_waves_per_simd<R>() / 2, (int)((160 * 1024) / (lds + 1024))));
    const int grid = std::min(cu_count() * per_cu, nitems);
    if (grid < 1) return hipSuccess;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kRingThreads), lds, s, dxf, items, nitems, queue, t.Zs, rec,
                       (int)rec_bytes, cs, outs);
    return hipGetLastError();
}

}  // namespace hpnfft
