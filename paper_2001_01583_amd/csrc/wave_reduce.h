// Cross-lane sums over a 64-lane wavefront for gfx950.
//
// The interpolation feeds the per-lane partials of consecutive points through
// halving steps: each exchange sends half of the pending values to the
// partner lanes and adds the other half, so 8 points cost about 7
// exchange-adds per component plus one 8-lane sum, instead of 8 full 6-step
// reductions.  Exchanges across 32- and 16-lane halves use gfx950's
// v_permlane32_swap / v_permlane16_swap; exchanges within a 16-lane row use
// DPP.
#pragma once

#include <hip/hip_runtime.h>

namespace hpnfft {

// ---- 32-bit lane moves -----------------------------------------------------

template <int CTRL>
__device__ inline unsigned dpp_u32(unsigned v)
{
    return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, true);
}

// Lane words of a value of type R (float: 1, double: 2).
template <typename R> struct Words;
template <> struct Words<float> {
    static constexpr int n = 1;
    __device__ static inline void split(float v, unsigned *w) { w[0] = __float_as_uint(v); }
    __device__ static inline float join(const unsigned *w) { return __uint_as_float(w[0]); }
};
template <> struct Words<double> {
    static constexpr int n = 2;
    __device__ static inline void split(double v, unsigned *w)
    {
        unsigned long long b = (unsigned long long)__double_as_longlong(v);
        w[0] = (unsigned)b;
        w[1] = (unsigned)(b >> 32);
    }
    __device__ static inline double join(const unsigned *w)
    {
        return __longlong_as_double((long long)(((unsigned long long)w[1] << 32) | w[0]));
    }
};

template <int CTRL, typename R>
__device__ inline R dpp(R v)
{
    unsigned w[Words<R>::n];
    Words<R>::split(v, w);
#pragma unroll
    for (int i = 0; i < Words<R>::n; ++i) w[i] = dpp_u32<CTRL>(w[i]);
    return Words<R>::join(w);
}

// (a, b) -> (lo halves of a and b, hi halves of a and b): after the swap the
// first result holds a's lanes 0-31 and b's lanes 0-31 (in lanes 32-63), the
// second a's lanes 32-63 (in lanes 0-31) and b's lanes 32-63.
template <typename R>
__device__ inline void swap32(R &a, R &b)
{
    unsigned wa[Words<R>::n], wb[Words<R>::n];
    Words<R>::split(a, wa);
    Words<R>::split(b, wb);
#pragma unroll
    for (int i = 0; i < Words<R>::n; ++i) {
        auto r = __builtin_amdgcn_permlane32_swap(wa[i], wb[i], false, false);
        wa[i] = r[0];
        wb[i] = r[1];
    }
    a = Words<R>::join(wa);
    b = Words<R>::join(wb);
}

// Same for 16-lane rows: the first result holds a's even rows in even rows
// and b's even rows in odd rows; the second a's odd rows and b's odd rows.
template <typename R>
__device__ inline void swap16(R &a, R &b)
{
    unsigned wa[Words<R>::n], wb[Words<R>::n];
    Words<R>::split(a, wa);
    Words<R>::split(b, wb);
#pragma unroll
    for (int i = 0; i < Words<R>::n; ++i) {
        auto r = __builtin_amdgcn_permlane16_swap(wa[i], wb[i], false, false);
        wa[i] = r[0];
        wb[i] = r[1];
    }
    a = Words<R>::join(wa);
    b = Words<R>::join(wb);
}

// Sum within aligned groups of 8 lanes; every lane of the group receives the
// group total.
template <typename R>
__device__ inline R sum8(R v)
{
    v += dpp<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp<0x141>(v);  // row_half_mirror
    return v;
}
// Halving steps for a stream of per-lane partials, one value per point.
// halve32(a, b): lanes 0-31 hold a summed over lanes l and l^32, lanes 32-63
// the same for b.
template <typename R>
__device__ inline R halve32(R a, R b)
{
    swap32(a, b);
    return a + b;
}
// halve16(a, b) for a = [p | q] and b = [p' | q'] (halves as left by
// halve32): rows 0..3 hold p, p', q, q', each summed over its four rows' lanes.
template <typename R>
__device__ inline R halve16(R a, R b)
{
    swap16(a, b);
    return a + b;
}
// Last step for a with rows (v0, v2, v1, v3) and b with rows (v4, v6, v5, v7)
// as left by halve16: the 8-lane group j receives the full sum of value
// v[bitrev3(j)] (groups: v0 v4 v2 v6 v1 v5 v3 v7).
template <typename R>
__device__ inline R halve8_sum(R a, R b)
{
    const bool hi = (threadIdx.x & 8) != 0;
    R t = hi ? b : a;
    R u = hi ? a : b;
    t += dpp<0x128>(u);  // row_ror:8
    return sum8(t);
}

}  // namespace hpnfft
