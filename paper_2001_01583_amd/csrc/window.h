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

// ---------------------------------------------------------------------------
// The window family of the precision experiment (Section 4 names the
// Gaussian, cardinal B-spline, sinc-power and Kaiser-Bessel windows).  Their
// formulas follow the NFFT literature (Potts, Steidl and Tasche 2001; Keiner,
// Kunis and Potts 2009), in grid units t = n x - l, each normalised to
// phi(0) = 1, truncated to |t| <= m, with divisor D(k) = the continuous
// Fourier transform of that normalised window at frequency k / n (cycles per
// cell), which is what the Scaling step divides by:
//   Gaussian     phi = exp(-t^2 / g),  g = 2 sigma m / ((2 sigma - 1) pi),
//                D(k) = sqrt(pi g) exp(-g (pi k / n)^2)
//   B-spline     phi = M_2m(t) / M_2m(0)  (centred cardinal B-spline of order
//                2m, support [-m, m]),  D(k) = sinc(pi k / n)^2m / M_2m(0)
//   sinc-power   phi = sinc(beta t)^2m,  beta = pi (2 sigma - 1) / (2 m sigma),
//                D(k) = (pi / beta) M_2m(pi k / (n beta))
//   Kaiser-Bessel  as above (kb_phi, kb_phihat).
// sinc(x) = sin(x) / x.
enum WindowKind { W_KAISER_BESSEL = 0, W_GAUSSIAN = 1, W_BSPLINE = 2, W_SINC_POWER = 3 };
constexpr int kMaxWindowM = 15;

struct WindowParams {
    int kind, m;
    double sigma;
    double b;         // Kaiser-Bessel shape, Gaussian g, or sinc-power beta
    double inv_peak;  // 1 / (unnormalised phi(0)): Kaiser-Bessel and B-spline
};

// Centred cardinal B-spline M_p(t) (support [-p/2, p/2]) and its derivative,
// by the two-term recursion
//   M_q(t) = ((q/2 + t) M_{q-1}(t + 1/2) + (q/2 - t) M_{q-1}(t - 1/2)) / (q - 1)
// evaluated bottom-up on the half-integer shifts t + s/2 (no cancellation:
// every term is non-negative).  p <= 2 kMaxWindowM.
HPNFFT_HD void bspline_eval(int p, double t, double *val, double *der)
{
    // level q holds M_q(t + (p - q) / 2 - j) for j = 0 .. p - q
    double a[2 * kMaxWindowM + 1];
    for (int j = 0; j <= p - 1; ++j) {
        const double u = t + 0.5 * (p - 1) - j;
        a[j] = (u >= -0.5 && u < 0.5) ? 1.0 : 0.0;
    }
    double dlast = 0.0;
    for (int q = 2; q <= p; ++q) {
        if (q == p) dlast = a[0] - a[1];  // M_p' = M_{p-1}(t + 1/2) - M_{p-1}(t - 1/2)
        for (int j = 0; j <= p - q; ++j) {
            const double u = t + 0.5 * (p - q) - j;
            a[j] = ((0.5 * q + u) * a[j] + (0.5 * q - u) * a[j + 1]) / (q - 1);
        }
    }
    *val = a[0];
    if (der) *der = p >= 2 ? dlast : 0.0;
}

HPNFFT_HD double sincd(double x) { return fabs(x) < 1e-8 ? 1.0 - x * x / 6.0 : sin(x) / x; }

// Normalised window and its derivative d phi / dt at distance t (0 beyond m).
HPNFFT_HD void win_eval(const WindowParams &w, double t, double *phi, double *dphi)
{
    const int m = w.m;
    if (fabs(t) > (double)m * (1.0 + 1e-12)) {
        *phi = 0.0;
        if (dphi) *dphi = 0.0;
        return;
    }
    switch (w.kind) {
    case W_GAUSSIAN: {
        const double v = exp(-t * t / w.b);
        *phi = v;
        if (dphi) *dphi = -2.0 * t / w.b * v;
        return;
    }
    case W_BSPLINE: {
        double v, d;
        bspline_eval(2 * m, t, &v, &d);
        *phi = v * w.inv_peak;
        if (dphi) *dphi = d * w.inv_peak;
        return;
    }
    case W_SINC_POWER: {
        const double x = w.b * t;
        const double sc = sincd(x);
        double p1 = 1.0;  // sinc^(2m - 1)
        for (int i = 0; i < 2 * m - 1; ++i) p1 *= sc;
        *phi = p1 * sc;
        if (dphi) {
            // d/dx sinc(x) = (x cos x - sin x) / x^2, ~ -x/3 near 0
            const double ds = fabs(x) < 1e-4 ? -x / 3.0 : (x * cos(x) - sin(x)) / (x * x);
            *dphi = 2.0 * m * p1 * ds * w.b;
        }
        return;
    }
    default:
        *phi = kb_phi(t, m, w.b, w.inv_peak);
        if (dphi) *dphi = kb_dphi(t, m, w.b, w.inv_peak);
        return;
    }
}

// Parameters of a window of the family for cut-off m and oversampling sigma.
inline WindowParams window_params(int kind, int m, double sigma)
{
    WindowParams w{kind, m, sigma, 0.0, 1.0};
    switch (kind) {
    case W_GAUSSIAN: w.b = 2.0 * sigma * m / ((2.0 * sigma - 1.0) * M_PI); break;
    case W_BSPLINE: {
        double v;
        bspline_eval(2 * m, 0.0, &v, nullptr);
        w.inv_peak = 1.0 / v;
        break;
    }
    case W_SINC_POWER: w.b = M_PI * (2.0 * sigma - 1.0) / (2.0 * m * sigma); break;
    default:
        w.b = kb_shape(sigma);
        w.inv_peak = 1.0 / kb_peak(m, w.b);
        break;
    }
    return w;
}

// Divisor D(k) of the Scaling step on a grid of n cells (host only).
inline double window_phihat(const WindowParams &w, long k, long n)
{
    const double x = M_PI * (double)k / (double)n;
    switch (w.kind) {
    case W_GAUSSIAN: return sqrt(M_PI * w.b) * exp(-w.b * x * x);
    case W_BSPLINE: {
        const double sc = sincd(x);
        double v = w.inv_peak;
        for (int i = 0; i < 2 * w.m; ++i) v *= sc;
        return v;
    }
    case W_SINC_POWER: {
        double v;
        bspline_eval(2 * w.m, x / w.b, &v, nullptr);
        return M_PI / w.b * v;
    }
    default: return kb_phihat(k, n, w.m, w.b, w.inv_peak);
    }
}

// A-priori bound E(m, sigma) of the one-dimensional approximation error of
// the gridding scheme, |approximate - exact| <= E ||f||_1 for every output,
// from the NFFT literature (Potts, Steidl and Tasche 2001, error estimates
// of the window family):
//   Kaiser-Bessel  4 pi (sqrt(m) + m) (1 - 1/sigma)^(1/4) exp(-2 pi m sqrt(1 - 1/sigma))
//   Gaussian       4 exp(-m pi (1 - 1/(2 sigma - 1)))
//   B-spline       4 (1 / (2 sigma - 1))^(2m)
//   sinc-power     (2 / sigma^(2m) + (sigma / (2 sigma - 1))^(2m)) / (m - 1),  m >= 2
// (host only; 4 for sinc-power at m = 1, where no bound is stated).
inline double window_error_bound(int kind, int m, double sigma)
{
    switch (kind) {
    case W_GAUSSIAN: return 4.0 * exp(-m * M_PI * (1.0 - 1.0 / (2.0 * sigma - 1.0)));
    case W_BSPLINE: return 4.0 * pow(1.0 / (2.0 * sigma - 1.0), 2.0 * m);
    case W_SINC_POWER:
        if (m < 2) return 4.0;
        return (2.0 / pow(sigma, 2.0 * m) + pow(sigma / (2.0 * sigma - 1.0), 2.0 * m)) / (m - 1.0);
    default:
        return 4.0 * M_PI * (sqrt((double)m) + m) * pow(1.0 - 1.0 / sigma, 0.25) *
               exp(-2.0 * M_PI * m * sqrt(1.0 - 1.0 / sigma));
    }
}

}  // namespace hpnfft
