// Spread and interpolation launchers for windows of 2m <= 16 cells (m <= 8);
// wider windows (m = 9 .. 15) are instantiated in k_spread_wide.hip.  The
// kernels themselves are in sweep.h.
#include "lines.h"
#include "ring.h"

namespace hpnfft {

template <typename R>
hipError_t launch_spread_wide(int m, const Xform *dxf, const SItem *items, int nitems, int *queue, Tiling t,
                              const unsigned char *rec, size_t rec_bytes, const R *fs, const int *cell_start,
                              hipStream_t s);
template <typename R>
hipError_t launch_interp_wide(int m, bool grad, const Xform *dxf, const SItem *items, int nitems, int *queue,
                              Tiling t, const unsigned char *rec, size_t rec_bytes, const int *cs, R *outs,
                              hipStream_t s);
template <typename R>
hipError_t launch_spread(int m, const Xform *dxf, const SItem *items, int nitems, int *queue, Tiling t,
                         const unsigned char *rec, size_t rec_bytes, const R *fs, const int *cell_start,
                         hipStream_t s)
{
#define HPNFFT_SPREAD_CASE(MM) \
    case MM: return spread_m<R, 2 * MM>(dxf, items, nitems, queue, t, rec, rec_bytes, fs, cell_start, s);
    if (m == 4 && t.ring && ring_tiling(8, t.T, t.Zs))
        return spread_ring<R>(dxf, items, nitems, queue, t, rec, rec_bytes, fs, cell_start, s);
    switch (m) {
        HPNFFT_SPREAD_CASE(1)
        HPNFFT_SPREAD_CASE(2)
        HPNFFT_SPREAD_CASE(3)
        HPNFFT_SPREAD_CASE(4)
        HPNFFT_SPREAD_CASE(5)
        HPNFFT_SPREAD_CASE(6)
        HPNFFT_SPREAD_CASE(7)
        HPNFFT_SPREAD_CASE(8)
    default: return launch_spread_wide<R>(m, dxf, items, nitems, queue, t, rec, rec_bytes, fs, cell_start, s);
    }
#undef HPNFFT_SPREAD_CASE
}

template <typename R>
hipError_t launch_interp(int m, bool grad, const Xform *dxf, const SItem *items, int nitems, int *queue,
                         Tiling t, const unsigned char *rec, size_t rec_bytes, const int *cs, R *outs,
                         hipStream_t s)
{
    if (m == 4 && !grad && t.ring && ring_tiling(8, t.T, t.Zs))
        return interp_ring<R>(dxf, items, nitems, queue, t, rec, rec_bytes, cs, outs, s);
#define HPNFFT_INTERP_CASE(MM)                                                                        \
    case MM:                                                                                          \
        return grad ? interp_m<R, 2 * MM, true>(dxf, items, nitems, queue, t, rec, rec_bytes, cs, outs, s) \
                    : interp_m<R, 2 * MM, false>(dxf, items, nitems, queue, t, rec, rec_bytes, cs, outs, s);
    switch (m) {
        HPNFFT_INTERP_CASE(1)
        HPNFFT_INTERP_CASE(2)
        HPNFFT_INTERP_CASE(3)
        HPNFFT_INTERP_CASE(4)
        HPNFFT_INTERP_CASE(5)
        HPNFFT_INTERP_CASE(6)
        HPNFFT_INTERP_CASE(7)
        HPNFFT_INTERP_CASE(8)
    default: return launch_interp_wide<R>(m, grad, dxf, items, nitems, queue, t, rec, rec_bytes, cs, outs, s);
    }
#undef HPNFFT_INTERP_CASE
}

template <typename R>
hipError_t launch_interp_lines(int m, const Xform *xf, const int n[3], int *queue, int T, const unsigned char *rec,
                               size_t rec_bytes, const int *cs, R *outs, hipStream_t s)
{
    if (m != 8) return hipErrorInvalidValue;
    return interp_lines_m<R, 16>(xf, n, queue, T, rec, rec_bytes, cs, outs, s);
}

template hipError_t launch_interp_lines<double>(int, const Xform *, const int *, int *, int, const unsigned char *,
                                                size_t, const int *, double *, hipStream_t);
template hipError_t launch_interp_lines<float>(int, const Xform *, const int *, int *, int, const unsigned char *,
                                               size_t, const int *, float *, hipStream_t);
template hipError_t launch_spread<double>(int, const Xform *, const SItem *, int, int *, Tiling,
                                          const unsigned char *, size_t, const double *, const int *, hipStream_t);
template hipError_t launch_spread<float>(int, const Xform *, const SItem *, int, int *, Tiling,
                                         const unsigned char *, size_t, const float *, const int *, hipStream_t);
template hipError_t launch_interp<double>(int, bool, const Xform *, const SItem *, int, int *, Tiling,
                                          const unsigned char *, size_t, const int *, double *, hipStream_t);
template hipError_t launch_interp<float>(int, bool, const Xform *, const SItem *, int, int *, Tiling,
                                         const unsigned char *, size_t, const int *, float *, hipStream_t);

}  // namespace hpnfft
