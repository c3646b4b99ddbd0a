// Interpolation by groups of single z-lines (the Interpolating step of
// Algorithm 5, Section 3).  Written for windows of 2m = 10 .. 16 cells; the
// plan selects it for 2m = 16, where it beats the staged sweep.
//
// A work item is a group of neighbouring z-lines (2 x 2, or a row of three
// for the widest float64 windows) and a slab of Zi planes along dim 0 (a
// multiple of 2m).  Each point is evaluated once, by
// the slab that holds its first tap plane.  A line's (2m)^2 tap rows are
// spread over NRG wavefronts of 64 lanes (lane <-> one (dy, dx) row), and
// each wavefront owns one (line, row group) for the whole slab: its register
// window of 2m complex values along dim 0 carries from plane to plane.  The
// planes reach the window through an LDS ring that holds one phase of 2m
// planes of the group's footprint ((2m + 1)^2 or 2m (2m + 2) cells): per phase all threads
// store the phase's planes (read from the grid into registers while the
// previous phase was swept), and after a barrier each wavefront takes one
// step per plane q: plane q enters slot q mod 2m, then the points whose
// window starts at q - 2m + 1 are evaluated.  The per-lane partials of
// consecutive points go through the halving steps of wave_reduce.h, and
// every 64 points each lane adds one point's row-group sum to the output
// (NRG adds per point, so the output is cleared first).
//
// Against the staged sweep this drops the z-halo (a point is evaluated once
// instead of by both slabs its window reaches), the record staging and its
// barriers, and the LDS tile of the slab: the per-point values the lanes
// share come through scalar loads straight from the records.
#pragma once

#include "sweep.h"

namespace hpnfft {

constexpr int kLinesZ = 64;  // slab depth target (planes), rounded down to a multiple of 2m

template <int M2> constexpr int lines_nrg() { return (M2 * M2 + 63) / 64; }
// Lines per group along dims 1 (GY) and 2 (GX).  2 x 2 in general; a row of
// three lines for float64 windows of 2m >= 14, whose 2m-slot float64 window
// takes 4 * 2m registers per lane: twelve wavefronts per workgroup leave 168
// registers per lane, enough to keep the next point's and the next phase's
// loads in flight.
template <typename R, int M2> struct LineGroup {
    static constexpr bool wide = sizeof(R) == 8 && M2 >= 14;
    static constexpr int GY = wide ? 1 : 2, GX = wide ? 3 : 2;
    static constexpr int PY = M2 + GY - 1, PX = M2 + GX - 1;  // footprint rows and columns
    static constexpr int threads = GY * GX * lines_nrg<M2>() * 64;
    static constexpr size_t lds = (size_t)M2 * PY * PX * 2 * sizeof(R);
};
__host__ __device__ constexpr int lines_slab(int M2) { return (kLinesZ / M2) * M2; }

template <typename R, int M2>
__global__ __launch_bounds__((LineGroup<R, M2>::threads)) void k_interp_lines(
    const Xform *__restrict__ xf, int nitems, int *__restrict__ queue, int T, const unsigned char *__restrict__ rec,
    int rbytes, const int *__restrict__ cell_start, R *__restrict__ outs)
{
    constexpr int m = M2 / 2;
    constexpr int NRG = lines_nrg<M2>();
    using G = LineGroup<R, M2>;
    constexpr int GY = G::GY, GX = G::GX, PX = G::PX;
    constexpr int PLANE = G::PY * PX;
    constexpr int NTH = G::threads;
    constexpr int NPF = (M2 * PLANE + NTH - 1) / NTH;  // ring cells per thread and phase
    constexpr int Zi = lines_slab(M2);
    extern __shared__ uint4 smem16[];
    R *ring = reinterpret_cast<R *>(smem16);  // [slot][footprint row][column] complex
    __shared__ int s_item;
    const int tid = threadIdx.x, lane = tid & 63, wave = uni(tid >> 6);
    const int line = wave / NRG, rg = wave - line * NRG;
    const int ly = line / GX, lx = line % GX;
    const int row = rg * 64 + lane;
    const bool active = row < M2 * M2;
    const int dy = active ? row / M2 : 0, dx = active ? row % M2 : 0;
    const int cell = (ly + dy) * PX + lx + dx;  // lane's cell in a ring plane
    // batch position whose sum this lane receives (see halve8_sum)
    const int j8 = lane >> 3;
    const int own = (lane & 7) * 8 + (((j8 & 1) << 2) | (j8 & 2) | (j8 >> 2));

    const int n0 = xf->n[0], n1 = xf->n[1], n2 = xf->n[2];
    const int ntx = xf->ntx;
    const int ngx = (n2 + GX - 1) / GX, ngy = (n1 + GY - 1) / GY;
    const long long poff = xf->poff;
    const int Mx = (int)xf->M;
    const unsigned char *recb = rec + (size_t)poff * rbytes;
    const gptr<const R> grid = as_global(reinterpret_cast<const R *>(xf->grid));
    const size_t pstride = (size_t)n1 * n2;

    struct PointData {
        R wz[M2];
        R wy, wx;
    };
    auto fetch = [&](const unsigned char *rp, PointData &d) __attribute__((always_inline)) {
        const cptr<R> pc = as_const(reinterpret_cast<const R *>(rp));
#pragma unroll
        for (int s = 0; s < M2; ++s) d.wz[s] = pc[s];
        const R *ps = reinterpret_cast<const R *>(rp);
        d.wy = ps[M2 + dy];
        d.wx = ps[2 * M2 + dx];
    };

    for (int it = next_item(queue, &s_item); it < nitems; it = next_item(queue, &s_item)) {
        const int gx = it % ngx, r0 = it / ngx;
        const int gy = r0 % ngy, sl = r0 / ngy;
        const int z0 = sl * Zi, zs = min(Zi, n0 - z0);
        const int Y0 = gy * GY, X0 = gx * GX;
        const int y = Y0 + ly, x = X0 + lx;
        const bool mine = y < n1 && x < n2;
        // the line's points by plane: key (tile, row and column in the
        // tile, plane) of the counting sort, whose tiles have edge T
        const int q1 = y / T, q2 = x / T;
        const int key_line = ((q1 * ntx + q2) * T + (y - q1 * T)) * T + (x - q2 * T);
        const int *cs = cell_start + xf->key_off + (long long)key_line * n0;
        auto plane_c = [&](int b) __attribute__((always_inline)) {
            int c = b + (m - 1) + z0;  // within [m - 1, 2 n0)
            c -= c >= n0 ? n0 : 0;
            return c;
        };

        PointData cur{};
        int cidx = -1;
        // partial sums of the last point evaluated, not yet reduced
        R pvr = 0, pvi = 0;
        int pend = -1;  // its sorted index (-1: none)
        const unsigned char *rcur = recb;
        R gr[M2], gi[M2];

        // halving-step state: partials of the open pair, quad and octet
        R s0r = 0, s0i = 0, s1r = 0, s1i = 0, s2r = 0, s2i = 0, orr = 0, ori = 0;
        int t = 0;    // position of the next point in the batch of 64
        int bsp = 0;  // lane t: sorted index of batch point t
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
        // every lane that holds the row-group sum of a point adds it to the
        // point's output (positions padded with zeros hold no point)
        auto drain = [&]() __attribute__((always_inline)) {
            const int count = t;
            while (t & 7) feed(R(0), R(0));
            const int sp_own = __builtin_amdgcn_ds_bpermute(own << 2, bsp);
            if (own < count) {
                __hip_atomic_fetch_add(&outs[(size_t)sp_own * 2], orr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_add(&outs[(size_t)sp_own * 2 + 1], ori, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
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
            rlo = cs[c];
            rhi = cs[c + 1];
        }
        const int zr = zs + M2 - 1;  // window planes of the slab's points
        // step q: plane q (slot k = q mod 2m) enters from the ring (planes
        // past the windows hold zeros); then the points whose window starts
        // at q - 2m + 1
        auto step = [&](const int k, const int q) __attribute__((always_inline)) {
            {
                const int o = (k * PLANE + cell) * 2;
                gr[k] = ring[o];
                gi[k] = ring[o + 1];
            }
            const int b = q - (M2 - 1);
            if (b >= 0 && b < zs) {
                const int pa = __builtin_amdgcn_readlane(rlo, b), pb = __builtin_amdgcn_readlane(rhi, b);
                for (int sp = pa; sp < pb; ++sp) {
                    // the previous point's reduction runs first, so that the
                    // loads of this point (issued after the previous point's
                    // sums, into the same registers: two sets of the shared
                    // weights do not fit the scalar registers of the widest
                    // windows) are in flight meanwhile
                    if (pend >= 0) reduce_pending();
                    if (sp != cidx) {
                        rcur = recb + (size_t)sp * rbytes;
                        fetch(rcur, cur);
                    }
                    R ar = 0, ai = 0;
#pragma unroll
                    for (int s = 0; s < M2; ++s) {
                        ar = fma(gr[s], cur.wz[s], ar);
                        ai = fma(gi[s], cur.wz[s], ai);
                    }
                    const R w12 = active ? cur.wy * cur.wx : R(0);
                    pvr = ar * w12;
                    pvi = ai * w12;
                    pend = sp;
                    const bool adv = sp + 1 < Mx;
                    rcur = adv ? rcur + rbytes : rcur;
                    fetch(rcur, cur);
                    cidx = adv ? sp + 1 : sp;
                }
            }
        };

        // ring cells of a phase, read from the grid one phase ahead
        R pr[NPF], pim[NPF];
        auto ring_fetch = [&](int ph) __attribute__((always_inline)) {
#pragma unroll
            for (int u = 0; u < NPF; ++u) {
                const int e = tid + u * NTH;
                const int zz = e / PLANE, c = e - zz * PLANE;
                const int q = ph * M2 + zz;
                pr[u] = pim[u] = R(0);
                if (e < M2 * PLANE && q < zr) {
                    const int fy = c / PX, fx = c - fy * PX;
                    int gz = z0 + q;  // below 2 n0
                    gz -= gz >= n0 ? n0 : 0;
                    int gyy = Y0 + fy - (m - 1), gxx = X0 + fx - (m - 1);
                    gyy += gyy < 0 ? n1 : 0;
                    gyy -= gyy >= n1 ? n1 : 0;
                    gyy -= gyy >= n1 ? n1 : 0;
                    gxx += gxx < 0 ? n2 : 0;
                    gxx -= gxx >= n2 ? n2 : 0;
                    gxx -= gxx >= n2 ? n2 : 0;
                    const size_t gidx = ((size_t)gz * pstride + (size_t)gyy * n2 + gxx) * 2;
                    pr[u] = grid[gidx];
                    pim[u] = grid[gidx + 1];
                }
            }
        };

        const int nph = (zr + M2 - 1) / M2;
        ring_fetch(0);
        for (int ph = 0; ph < nph; ++ph) {
            if (ph > 0) __syncthreads();  // the previous phase's steps have read the ring
#pragma unroll
            for (int u = 0; u < NPF; ++u) {
                const int e = tid + u * NTH;
                if (e < M2 * PLANE) {
                    ring[2 * e] = pr[u];
                    ring[2 * e + 1] = pim[u];
                }
            }
            __syncthreads();
            if (ph + 1 < nph) ring_fetch(ph + 1);
            if (mine) {
#pragma unroll
                for (int k = 0; k < M2; ++k) step(k, ph * M2 + k);
            }
        }
        if (mine && pend >= 0) reduce_pending();
        if (mine && t > 0) drain();
    }
    release_queue(queue);
}

// One launch per transform (the items of a transform are its line groups
// times its slabs).  xf: the transform's device descriptor; n: its grid
// edges on the host.
template <typename R, int M2>
static hipError_t interp_lines_m(const Xform *xf, const int n[3], int *queue, int T, const unsigned char *rec,
                                 size_t rec_bytes, const int *cs, R *outs, hipStream_t s)
{
    const int nsl = (n[0] + lines_slab(M2) - 1) / lines_slab(M2);
    using G = LineGroup<R, M2>;
    const int nitems = nsl * ((n[1] + G::GY - 1) / G::GY) * ((n[2] + G::GX - 1) / G::GX);
    constexpr size_t lds = G::lds;
    auto kern = k_interp_lines<R, M2>;
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const int grid = std::min(cu_count(), nitems);
    if (grid < 1) return hipSuccess;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(G::threads), lds, s, xf, nitems, queue, T, rec,
                       (int)rec_bytes, cs, outs);
    return hipGetLastError();
}

}  // namespace hpnfft
