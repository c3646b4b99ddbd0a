// Kaiser-Bessel window of the gridding scheme (Section 2 of the paper names
// the window family; Section 4 lists KAISER_BESSEL among the four windows it
// evaluates).  The formulas follow the standard NFFT form of this window
// (Potts, Steidl and Tasche 2001; Keiner, Kunis and Potts 2009):
//
//   grid units t = n x - l, cut-off m, shape b = pi (2 - 1/sigma),
//   Phi(t)    = sinh(b r) / (pi r),  r = sqrt(m^2 - t^2),  |t| <= m,  0 beyond,
//   PhiHat(k) = I0(m sqrt(b^2 - (2 pi k / n)^2))  for |k| <= n/(2 sigma),
//
// so that the periodised window has Fourier coefficients c_k = PhiHat(k) on
// the oversampled grid.  Everything is divided by Phi(0) = sinh(b m)/(pi m)
// so that values stay O(1) in float32 for any m.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace hpnfft {

#define HPNFFT_HD __host__ __device__ inline

HPNFFT_HD double kb_shape(double sigma) { return M_PI * (2.0 - 1.0 / sigma); }

// Phi(0) for the normalisation.
HPNFFT_HD double kb_peak(int m, double b) { return sinh(b * m) / (M_PI * m); }

// sinh(x)/x and (x cosh x - sinh x)/x^3 for x >= 0: power series below
// x = 0.5 (ten terms, truncation below 1e-21 relative), else one exp.
HPNFFT_HD double sinhc(double x)
{
    if (x < 0.5) {
        const double z2 = x * x;
        double term = 1.0, acc = 1.0;
        for (int k = 1; k <= 9; ++k) {
            term *= z2 / ((2.0 * k) * (2.0 * k + 1.0));
            acc += term;
        }
        return acc;
    }
    const double e = exp(x);
    return 0.5 * (e - 1.0 / e) / x;
}
HPNFFT_HD double sinhc_d(double x)
{
    if (x < 0.5) {
        // sum_{k>=1} x^(2k-2) * 2k / (2k+1)!
        const double z2 = x * x;
        double term = 1.0, acc = 0.0, fact = 6.0;
        for (int k = 1; k <= 10; ++k) {
            acc += term * (2.0 * k) / fact;
            term *= z2;
            fact *= (2.0 * k + 2.0) * (2.0 * k + 3.0);
        }
        return acc;
    }
    const double e = exp(x), ei = 1.0 / e;
    return (0.5 * x * (e + ei) - 0.5 * (e - ei)) / (x * x * x);
}

// r = sqrt(m^2 - t^2), or -1 where |t| > m beyond rounding.
HPNFFT_HD double kb_radius(double t, int m)
{
    double r2 = (double)m * m - t * t;
    if (r2 < 0.0) {
        // |t| can exceed m only by rounding at the truncation edge.
        if (r2 < -1e-12 * m * m) return -1.0;
        r2 = 0.0;
    }
    return sqrt(r2);
}

// Normalised window value at grid-unit distance t:
// sinh(b r)/(pi r) = b sinhc(b r)/pi.
HPNFFT_HD double kb_phi(double t, int m, double b, double inv_peak)
{
    const double r = kb_radius(t, m);
    if (r < 0.0) return 0.0;
    return b * sinhc(b * r) * (1.0 / M_PI) * inv_peak;
}

// Normalised derivative dPhi/dt:
//   dPhi/dt = -t (b r cosh(b r) - sinh(b r)) / (pi r^3) = -t b^3 sinhc_d(b r) / pi.
HPNFFT_HD double kb_dphi(double t, int m, double b, double inv_peak)
{
    const double r = kb_radius(t, m);
    if (r < 0.0) return 0.0;
    return -t * b * b * b * sinhc_d(b * r) * (1.0 / M_PI) * inv_peak;
}

// Modified Bessel function I0 by its all-positive power series
// sum_k (z^2/4)^k / (k!)^2 (no cancellation; z <= m b <= 40 here).
inline double bessel_i0(double z)
{
    double y = 0.25 * z * z, term = 1.0, acc = 1.0;
    for (int k = 1; k < 500; ++k) {
        term *= y / ((double)k * (double)k);
        acc += term;
        if (term < 1e-18 * acc) break;
    }
    return acc;
}

// Normalised Fourier coefficient c_k of the periodised window on a grid of n
// cells (the "weight factor" of the Scaling step, Section 2).
inline double kb_phihat(long k, long n, int m, double b, double inv_peak)
{
    double w = 2.0 * M_PI * (double)k / (double)n;
    double a = b * b - w * w;
    if (a < 0.0) a = 0.0;  // only reachable for k outside I_N with sigma < 2
    return bessel_i0((double)m * sqrt(a)) * inv_peak;
}

}  // namespace hpnfft
