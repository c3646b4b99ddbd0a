// Spread and interpolation launchers for wide windows, 2m = 18 .. 30 cells
// (m = 9 .. 15: the upper part of the cut-off range of the precision
// experiment in Section 4).  Same kernels as k_spread.hip (sweep.h), compiled
// in their own translation unit so the two build in parallel.  These widths
// use single-line runs and 256-thread workgroups (a lane's register window
// holds 2m complex values).
#include "sweep.h"

namespace hpnfft {

template <typename R>
hipError_t launch_spread_wide(int m, const Xform *dxf, const SItem *items, int nitems, int *queue, Tiling t,
                              const unsigned char *rec, size_t rec_bytes, const R *fs, const int *cell_start,
                              hipStream_t s)
{
#define HPNFFT_SPREAD_CASE(MM) \
    case MM: return spread_m<R, 2 * MM>(dxf, items, nitems, queue, t, rec, rec_bytes, fs, cell_start, s);
    switch (m) {
        HPNFFT_SPREAD_CASE(9)
        HPNFFT_SPREAD_CASE(10)
        HPNFFT_SPREAD_CASE(11)
        HPNFFT_SPREAD_CASE(12)
        HPNFFT_SPREAD_CASE(13)
        HPNFFT_SPREAD_CASE(14)
        HPNFFT_SPREAD_CASE(15)
    default: return hipErrorInvalidValue;
    }
#undef HPNFFT_SPREAD_CASE
}

template <typename R>
hipError_t launch_interp_wide(int m, bool grad, const Xform *dxf, const SItem *items, int nitems, int *queue,
                              Tiling t, const unsigned char *rec, size_t rec_bytes, const int *cs, R *outs,
                              hipStream_t s)
{
#define HPNFFT_INTERP_CASE(MM)                                                                        \
    case MM:                                                                                          \
        return grad ? interp_m<R, 2 * MM, true>(dxf, items, nitems, queue, t, rec, rec_bytes, cs, outs, s) \
                    : interp_m<R, 2 * MM, false>(dxf, items, nitems, queue, t, rec, rec_bytes, cs, outs, s);
    switch (m) {
        HPNFFT_INTERP_CASE(9)
        HPNFFT_INTERP_CASE(10)
        HPNFFT_INTERP_CASE(11)
        HPNFFT_INTERP_CASE(12)
        HPNFFT_INTERP_CASE(13)
        HPNFFT_INTERP_CASE(14)
        HPNFFT_INTERP_CASE(15)
    default: return hipErrorInvalidValue;
    }
#undef HPNFFT_INTERP_CASE
}

template hipError_t launch_spread_wide<double>(int, const Xform *, const SItem *, int, int *, Tiling,
                                               const unsigned char *, size_t, const double *, const int *,
                                               hipStream_t);
template hipError_t launch_spread_wide<float>(int, const Xform *, const SItem *, int, int *, Tiling,
                                              const unsigned char *, size_t, const float *, const int *,
                                              hipStream_t);
template hipError_t launch_interp_wide<double>(int, bool, const Xform *, const SItem *, int, int *, Tiling,
                                               const unsigned char *, size_t, const int *, double *, hipStream_t);
template hipError_t launch_interp_wide<float>(int, bool, const Xform *, const SItem *, int, int *, Tiling,
                                              const unsigned char *, size_t, const int *, float *, hipStream_t);

}  // namespace hpnfft
