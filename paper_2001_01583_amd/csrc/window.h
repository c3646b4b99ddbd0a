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

// Normalised window value at grid-unit distance t.
HPNFFT_HD double kb_phi(double t, int m, double b, double inv_peak)
{
    double r2 = (double)m * m - t * t;
    if (r2 < 0.0) {
        // |t| can exceed m only by rounding at the truncation edge.
        if (r2 < -1e-12 * m * m) return 0.0;
        r2 = 0.0;
    }
    double r = sqrt(r2);
    double br = b * r;
    double v = (br < 1e-8) ? b * (1.0 + br * br / 6.0) : sinh(br) / r;
    return v * (1.0 / M_PI) * inv_peak;
}

// Normalised derivative dPhi/dt:
//   dPhi/dt = -t (b r cosh(b r) - sinh(b r)) / (pi r^3),
// with the series b^3/3 + b^5 r^2/30 + ... of (b r cosh - sinh)/r^3 near r = 0.
HPNFFT_HD double kb_dphi(double t, int m, double b, double inv_peak)
{
    double r2 = (double)m * m - t * t;
    if (r2 < 0.0) {
        if (r2 < -1e-12 * m * m) return 0.0;
        r2 = 0.0;
    }
    double r = sqrt(r2);
    double br = b * r;
    double q;  // (b r cosh(b r) - sinh(b r)) / r^3
    if (br < 0.5) {
        // sum_{k>=1} b^3 (br)^{2k-2} * 2k / (2k+1)!
        double z2 = br * br, term = 1.0, acc = 0.0;
        double fact = 6.0;  // (2k+1)! for k = 1
        for (int k = 1; k <= 10; ++k) {
            acc += term * (2.0 * k) / fact;
            term *= z2;
            fact *= (2.0 * k + 2.0) * (2.0 * k + 3.0);
        }
        q = b * b * b * acc;
    } else {
        q = (br * cosh(br) - sinh(br)) / (r2 * r);
    }
    return -t * q * (1.0 / M_PI) * inv_peak;
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
