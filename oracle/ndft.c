/*
 * Reference oracle for the nonequispaced discrete Fourier transform (NDFT).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * CPU definition that the GPU library is checked against.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load
 * it.  It shares no code, header, table or helper with the GPU library.
 *
 * Everything is IEEE double precision, no fast-math, deterministic: every
 * output is owned by one OpenMP thread and summed in index order with a
 * Neumaier-compensated sum, so results do not depend on the thread count.
 *
 * Paper: Yang & Wang, "A Hybrid MPI-CUDA Approach for Nonequispaced Discrete
 * Fourier Transformation" (arXiv 2001.01583).
 *   - frequency box I_N = { k : -N_t/2 <= k_t < N_t/2 }, domain [-1/2,1/2)^d
 *     (Section 1, the paragraph introducing I_N and Pi^d);
 *   - NDFT, Eq. (5):  fhat(k) = sum_j f_j exp(-2 pi i k.x_j),  k in I_N;
 *   - its transpose, Eq. (6):  f(x_j) = sum_k fhat(k) exp(+2 pi i k.x_j);
 *   - error metric, Eq. (9): relative l2 norm of the difference;
 *   - Ewald energy of Eqs. (10)-(12) (Section 5).
 *
 * Storage conventions (shared with the GPU library only as a documented
 * interface, not as code): row-major (C order), last dimension fastest;
 * frequency k is stored at index k_t + N_t/2 per dimension; complex values are
 * interleaved (re, im); points are M x d row-major.
 */
#include <math.h>
#include <omp.h>
#include <stddef.h>
#include <stdint.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ---------------------------------------------------------------------- */
/* Compensated (Neumaier) accumulator.                                     */
typedef struct { double s, c; } nsum;

static inline void nsum_add(nsum *a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else                       a->c += (v - t) + a->s;
    a->s = t;
}
static inline double nsum_get(const nsum *a) { return a->s + a->c; }

/* Fractional part of k*x, reduced to about [-1/2, 1/2], keeping the rounding
 * error of the product (fma gives it exactly) so the phase stays accurate to
 * a few ulp even for large k. */
static inline double frac_prod(double k, double x)
{
    double p = k * x;
    double e = fma(k, x, -p);          /* exact: k*x = p + e */
    double r = p - nearbyint(p);       /* exact for |p| < 2^52 */
    return r + e;
}

/* exp(sign * 2 pi i * phase) for phase given in cycles. */
static inline void cis_cycles(double phase, double sign, double *c, double *s)
{
    double a = 2.0 * M_PI * phase;
    *c = cos(a);
    *s = sign * sin(a);
}

/* Decode the linear index of a frequency in I_N (C order, centred storage)
 * into the integer frequency vector k. */
static inline void decode_k(int d, const int64_t *N, int64_t lin, double *k)
{
    for (int t = d - 1; t >= 0; --t) {
        int64_t it = lin % N[t];
        lin /= N[t];
        k[t] = (double)(it - N[t] / 2);
    }
}

static int64_t box_size(int d, const int64_t *N)
{
    int64_t s = 1;
    for (int t = 0; t < d; ++t) s *= N[t];
    return s;
}

/* ---------------------------------------------------------------------- */
/* Eq. (5): fhat(k) = sum_j f_j exp(-2 pi i k.x_j).                          */
/* kidx: nk linear indices into I_N (C order, centred), or NULL for all of   */
/* I_N (then nk must equal #I_N).  out: nk complex values.                   */
int oracle_ndft_adjoint(int d, const int64_t *N, int64_t M,
                        const double *x, const double *f,
                        int64_t nk, const int64_t *kidx, double *out)
{
    if (d < 1 || d > 3 || M < 0 || nk < 0) return -1;
    int64_t nall = box_size(d, N);
    if (!kidx && nk != nall) return -1;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < nk; ++q) {
        int64_t lin = kidx ? kidx[q] : q;
        double k[3] = {0, 0, 0};
        decode_k(d, N, lin, k);
        nsum re = {0, 0}, im = {0, 0};
        for (int64_t j = 0; j < M; ++j) {
            double ph = 0.0;
            for (int t = 0; t < d; ++t) ph += frac_prod(k[t], x[j * d + t]);
            double c, s;
            cis_cycles(ph, -1.0, &c, &s);
            double fr = f[2 * j], fi = f[2 * j + 1];
            nsum_add(&re, fr * c - fi * s);
            nsum_add(&im, fr * s + fi * c);
        }
        out[2 * q] = nsum_get(&re);
        out[2 * q + 1] = nsum_get(&im);
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Eq. (6): f(x_j) = sum_{k in I_N} fhat(k) exp(+2 pi i k.x_j).              */
/* jidx: nj point indices, or NULL for all points (nj must equal M).         */
int oracle_ndft_forward(int d, const int64_t *N, int64_t M,
                        const double *x, const double *fhat,
                        int64_t nj, const int64_t *jidx, double *out)
{
    if (d < 1 || d > 3 || M < 0 || nj < 0) return -1;
    if (!jidx && nj != M) return -1;
    int64_t nall = box_size(d, N);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < nj; ++q) {
        int64_t j = jidx ? jidx[q] : q;
        nsum re = {0, 0}, im = {0, 0};
        for (int64_t lin = 0; lin < nall; ++lin) {
            double k[3] = {0, 0, 0};
            decode_k(d, N, lin, k);
            double ph = 0.0;
            for (int t = 0; t < d; ++t) ph += frac_prod(k[t], x[j * d + t]);
            double c, s;
            cis_cycles(ph, +1.0, &c, &s);
            double ar = fhat[2 * lin], ai = fhat[2 * lin + 1];
            nsum_add(&re, ar * c - ai * s);
            nsum_add(&im, ar * s + ai * c);
        }
        out[2 * q] = nsum_get(&re);
        out[2 * q + 1] = nsum_get(&im);
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Gradient of a real loss L through Eq. (5).                                */
/* gbar(k) = dL/dRe fhat(k) + i dL/dIm fhat(k) for every k in I_N.           */
/* Differentiating Eq. (5):                                                  */
/*   d fhat(k) / d f_j       = exp(-2 pi i k.x_j)          (holomorphic),    */
/*   d fhat(k) / d x_{j,t}   = -2 pi i k_t f_j exp(-2 pi i k.x_j).           */
/* Hence, in the (dL/dRe + i dL/dIm) convention for the complex input f:     */
/*   grad_f_j    = sum_k gbar(k) exp(+2 pi i k.x_j),                         */
/*   grad_x_{j,t} = Re sum_k conj(gbar(k)) * (-2 pi i k_t f_j e^{-2pi i k.x_j}).*/
/* jidx selects nj points (NULL: all).  grad_f: nj complex; grad_x: nj x d.  */
int oracle_ndft_adjoint_grad(int d, const int64_t *N, int64_t M,
                             const double *x, const double *f,
                             const double *gbar,
                             int64_t nj, const int64_t *jidx,
                             double *grad_f, double *grad_x)
{
    if (d < 1 || d > 3 || M < 0 || nj < 0) return -1;
    if (!jidx && nj != M) return -1;
    int64_t nall = box_size(d, N);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < nj; ++q) {
        int64_t j = jidx ? jidx[q] : q;
        nsum gr = {0, 0}, gi = {0, 0};
        nsum gx[3] = {{0, 0}, {0, 0}, {0, 0}};
        double fr = f[2 * j], fi = f[2 * j + 1];
        for (int64_t lin = 0; lin < nall; ++lin) {
            double k[3] = {0, 0, 0};
            decode_k(d, N, lin, k);
            double ph = 0.0;
            for (int t = 0; t < d; ++t) ph += frac_prod(k[t], x[j * d + t]);
            double c, s;                       /* e = exp(-2 pi i k.x) = c + i s */
            cis_cycles(ph, -1.0, &c, &s);
            double br = gbar[2 * lin], bi = gbar[2 * lin + 1];
            /* gbar * conj(e) = gbar * exp(+2 pi i k.x) */
            nsum_add(&gr, br * c + bi * s);
            nsum_add(&gi, bi * c - br * s);
            /* f_j * e */
            double pr = fr * c - fi * s, pi_ = fr * s + fi * c;
            for (int t = 0; t < d; ++t) {
                /* -2 pi i k_t (pr + i pi_) = 2 pi k_t (pi_ - i pr) */
                double dr = 2.0 * M_PI * k[t] * pi_;
                double di = -2.0 * M_PI * k[t] * pr;
                /* Re(conj(gbar) * (dr + i di)) = br*dr + bi*di */
                nsum_add(&gx[t], br * dr + bi * di);
            }
        }
        grad_f[2 * q] = nsum_get(&gr);
        grad_f[2 * q + 1] = nsum_get(&gi);
        for (int t = 0; t < d; ++t) grad_x[q * d + t] = nsum_get(&gx[t]);
    }
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Ewald electrostatics, Eqs. (10)-(12), cubic box of side L, charges q.     */
/* Real-space part, Eq. (11): 1/2 sum_n' sum_{i,j} q_i q_j erfc(a r)/r,      */
/* r = |r_ij + n L|, the n = 0 term omitted for i = j; images |n_t| <= nsh.  */
/* Also returns the force F_i = -dU/dr_i (3 per ion) when forces != NULL.    */
double oracle_ewald_real(int64_t M, const double *r, const double *q,
                         double L, double alpha, int nsh, double *forces)
{
    double total = 0.0;
    const double two_over_sqrtpi = 2.0 / sqrt(M_PI);
#pragma omp parallel for schedule(dynamic, 8) reduction(+:total)
    for (int64_t i = 0; i < M; ++i) {
        nsum ui = {0, 0};
        nsum fx[3] = {{0, 0}, {0, 0}, {0, 0}};
        for (int64_t j = 0; j < M; ++j) {
            for (int a = -nsh; a <= nsh; ++a)
            for (int b = -nsh; b <= nsh; ++b)
            for (int c = -nsh; c <= nsh; ++c) {
                if (i == j && a == 0 && b == 0 && c == 0) continue;
                double dx = r[3 * i] - r[3 * j] + a * L;
                double dy = r[3 * i + 1] - r[3 * j + 1] + b * L;
                double dz = r[3 * i + 2] - r[3 * j + 2] + c * L;
                double rr = sqrt(dx * dx + dy * dy + dz * dz);
                double qq = q[i] * q[j];
                nsum_add(&ui, 0.5 * qq * erfc(alpha * rr) / rr);
                if (forces) {
                    /* -d/dr_i [q_i q_j erfc(a r)/r] summed over j, n (the 1/2 */
                    /* cancels the double counting of the pair).               */
                    double g = qq * (erfc(alpha * rr) / rr
                               + two_over_sqrtpi * alpha * exp(-alpha * alpha * rr * rr))
                               / (rr * rr);
                    nsum_add(&fx[0], g * dx);
                    nsum_add(&fx[1], g * dy);
                    nsum_add(&fx[2], g * dz);
                }
            }
        }
        total += nsum_get(&ui);
        if (forces)
            for (int t = 0; t < 3; ++t) forces[3 * i + t] = nsum_get(&fx[t]);
    }
    return total;
}

/* Reciprocal-space part, Eq. (12):                                          */
/*   1/(2 pi L) sum_{n != 0} exp(-pi^2 |n|^2/(a L)^2)/|n|^2 S(n) S(-n)       */
/*   - a/sqrt(pi) sum_i q_i^2,                                               */
/* with S(n) = sum_i q_i exp(-2 pi i n.r_i / L) over the cube |n_t| <= kmax. */
/* For real charges S(-n) = conj S(n), so S(n)S(-n) = |S(n)|^2.             */
double oracle_ewald_recip(int64_t M, const double *r, const double *q,
                          double L, double alpha, int kmax)
{
    int64_t side = 2 * (int64_t)kmax + 1;
    int64_t nk = side * side * side;
    double total = 0.0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+:total)
    for (int64_t lin = 0; lin < nk; ++lin) {
        int64_t n0 = lin / (side * side) - kmax;
        int64_t n1 = (lin / side) % side - kmax;
        int64_t n2 = lin % side - kmax;
        if (n0 == 0 && n1 == 0 && n2 == 0) continue;
        double n2sum = (double)(n0 * n0 + n1 * n1 + n2 * n2);
        double w = exp(-M_PI * M_PI * n2sum / (alpha * L * alpha * L)) / n2sum;
        nsum sr = {0, 0}, si = {0, 0};
        for (int64_t i = 0; i < M; ++i) {
            double ph = frac_prod((double)n0, r[3 * i] / L)
                      + frac_prod((double)n1, r[3 * i + 1] / L)
                      + frac_prod((double)n2, r[3 * i + 2] / L);
            double c, s;
            cis_cycles(ph, -1.0, &c, &s);
            nsum_add(&sr, q[i] * c);
            nsum_add(&si, q[i] * s);
        }
        double Sr = nsum_get(&sr), Si = nsum_get(&si);
        total += w * (Sr * Sr + Si * Si) / (2.0 * M_PI * L);
    }
    double self = 0.0;
    for (int64_t i = 0; i < M; ++i) self += q[i] * q[i];
    return total - alpha / sqrt(M_PI) * self;
}

/* Reciprocal-space forces, Eq. (12) differentiated.  S: caller scratch of   */
/* 2 * (2 kmax + 1)^3 doubles.  F_i = -(1/(2 pi L)) sum_n w(n)               */
/*   * 2 Re[conj(S(n)) (-2 pi i n_t / L) q_i exp(-2 pi i n.r_i/L)].          */
int oracle_ewald_recip_forces(int64_t M, const double *r, const double *q,
                              double L, double alpha, int kmax,
                              double *S, double *forces)
{
    int64_t side = 2 * (int64_t)kmax + 1;
    int64_t nk = side * side * side;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t lin = 0; lin < nk; ++lin) {
        int64_t n0 = lin / (side * side) - kmax;
        int64_t n1 = (lin / side) % side - kmax;
        int64_t n2 = lin % side - kmax;
        nsum sr = {0, 0}, si = {0, 0};
        for (int64_t i = 0; i < M; ++i) {
            double ph = frac_prod((double)n0, r[3 * i] / L)
                      + frac_prod((double)n1, r[3 * i + 1] / L)
                      + frac_prod((double)n2, r[3 * i + 2] / L);
            double c, s;
            cis_cycles(ph, -1.0, &c, &s);
            nsum_add(&sr, q[i] * c);
            nsum_add(&si, q[i] * s);
        }
        S[2 * lin] = nsum_get(&sr);
        S[2 * lin + 1] = nsum_get(&si);
    }
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t i = 0; i < M; ++i) {
        nsum fx[3] = {{0, 0}, {0, 0}, {0, 0}};
        for (int64_t lin = 0; lin < nk; ++lin) {
            int64_t nv[3];
            nv[0] = lin / (side * side) - kmax;
            nv[1] = (lin / side) % side - kmax;
            nv[2] = lin % side - kmax;
            if (nv[0] == 0 && nv[1] == 0 && nv[2] == 0) continue;
            double n2sum = (double)(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
            double w = exp(-M_PI * M_PI * n2sum / (alpha * L * alpha * L)) / n2sum;
            double ph = frac_prod((double)nv[0], r[3 * i] / L)
                      + frac_prod((double)nv[1], r[3 * i + 1] / L)
                      + frac_prod((double)nv[2], r[3 * i + 2] / L);
            double c, s;
            cis_cycles(ph, -1.0, &c, &s);        /* e = c + i s */
            double Sr = S[2 * lin], Si = S[2 * lin + 1];
            /* conj(S) e = (Sr c + Si s) + i (Sr s - Si c) */
            double pim = Sr * s - Si * c;        /* Im(conj(S) e) */
            for (int t = 0; t < 3; ++t) {
                /* Re[(-2 pi i n_t/L) q_i (pr + i pim)] = 2 pi n_t q_i pim / L */
                double dre = 2.0 * M_PI * (double)nv[t] * q[i] * pim / L;
                /* F = -dU/dr = -(1/(2 pi L)) w 2 dre */
                nsum_add(&fx[t], -w * 2.0 * dre / (2.0 * M_PI * L));
            }
        }
        for (int t = 0; t < 3; ++t) forces[3 * i + t] = nsum_get(&fx[t]);
    }
    return 0;
}

/* Eq. (12) energy and the forces of selected ions only, for lattices whose */
/* full force set is too costly to evaluate directly.  Same sums as the two  */
/* functions above: S(n) over the cube |n_t| <= kmax from all M ions (stored */
/* in S, 2 (2 kmax + 1)^3 doubles), the energy of Eq. (12) including the     */
/* self term, and F for the nsel ions listed in sel (forces: nsel x 3).      */
double oracle_ewald_recip_sel(int64_t M, const double *r, const double *q,
                              double L, double alpha, int kmax,
                              int64_t nsel, const int64_t *sel,
                              double *S, double *forces)
{
    int64_t side = 2 * (int64_t)kmax + 1;
    int64_t nk = side * side * side;
    double total = 0.0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+:total)
    for (int64_t lin = 0; lin < nk; ++lin) {
        int64_t n0 = lin / (side * side) - kmax;
        int64_t n1 = (lin / side) % side - kmax;
        int64_t n2 = lin % side - kmax;
        nsum sr = {0, 0}, si = {0, 0};
        for (int64_t i = 0; i < M; ++i) {
            double ph = frac_prod((double)n0, r[3 * i] / L)
                      + frac_prod((double)n1, r[3 * i + 1] / L)
                      + frac_prod((double)n2, r[3 * i + 2] / L);
            double c, s;
            cis_cycles(ph, -1.0, &c, &s);
            nsum_add(&sr, q[i] * c);
            nsum_add(&si, q[i] * s);
        }
        double Sr = nsum_get(&sr), Si = nsum_get(&si);
        S[2 * lin] = Sr;
        S[2 * lin + 1] = Si;
        if (n0 == 0 && n1 == 0 && n2 == 0) continue;
        double n2sum = (double)(n0 * n0 + n1 * n1 + n2 * n2);
        double w = exp(-M_PI * M_PI * n2sum / (alpha * L * alpha * L)) / n2sum;
        total += w * (Sr * Sr + Si * Si) / (2.0 * M_PI * L);
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t a = 0; a < nsel; ++a) {
        int64_t i = sel[a];
        nsum fx[3] = {{0, 0}, {0, 0}, {0, 0}};
        for (int64_t lin = 0; lin < nk; ++lin) {
            int64_t nv[3];
            nv[0] = lin / (side * side) - kmax;
            nv[1] = (lin / side) % side - kmax;
            nv[2] = lin % side - kmax;
            if (nv[0] == 0 && nv[1] == 0 && nv[2] == 0) continue;
            double n2sum = (double)(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
            double w = exp(-M_PI * M_PI * n2sum / (alpha * L * alpha * L)) / n2sum;
            double ph = frac_prod((double)nv[0], r[3 * i] / L)
                      + frac_prod((double)nv[1], r[3 * i + 1] / L)
                      + frac_prod((double)nv[2], r[3 * i + 2] / L);
            double c, s;
            cis_cycles(ph, -1.0, &c, &s);
            double pim = S[2 * lin] * s - S[2 * lin + 1] * c;
            for (int t = 0; t < 3; ++t) {
                double dre = 2.0 * M_PI * (double)nv[t] * q[i] * pim / L;
                nsum_add(&fx[t], -w * 2.0 * dre / (2.0 * M_PI * L));
            }
        }
        for (int t = 0; t < 3; ++t) forces[3 * a + t] = nsum_get(&fx[t]);
    }
    double self = 0.0;
    for (int64_t i = 0; i < M; ++i) self += q[i] * q[i];
    return total - alpha / sqrt(M_PI) * self;
}

/* Eq. (9): relative l2 error ||a - s|| / ||s|| over n complex values. */
double oracle_rel_l2(int64_t n, const double *a, const double *s)
{
    nsum num = {0, 0}, den = {0, 0};
    for (int64_t i = 0; i < 2 * n; ++i) {
        double dlt = a[i] - s[i];
        nsum_add(&num, dlt * dlt);
        nsum_add(&den, s[i] * s[i]);
    }
    return sqrt(nsum_get(&num) / nsum_get(&den));
}

/* Threads the OpenMP loops above run on (reported beside timings). */
int oracle_threads(void)
{
    int n = 1;
#pragma omp parallel
    {
#pragma omp single
        n = omp_get_num_threads();
    }
    return n;
}
