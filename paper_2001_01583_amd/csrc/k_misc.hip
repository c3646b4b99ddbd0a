// Small elementwise kernels: zero fill (used instead of memset so the
// sequences can be captured in a HIP graph), value gather into sorted point
// order, result scatter back to the caller's order, the gradient epilogue,
// and the reciprocal-space Ewald sum of Eq. (12) with a float64 reduction.
#include "internal.h"

namespace hpnfft {

__global__ void k_zero(uint4 *__restrict__ p, size_t n16, unsigned char *__restrict__ tail,
                       size_t ntail)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n16; i += stride) p[i] = make_uint4(0, 0, 0, 0);
    if (blockIdx.x == 0 && threadIdx.x < ntail) tail[threadIdx.x] = 0;
}

hipError_t launch_zero(void *p, size_t bytes, hipStream_t s)
{
    if (bytes == 0) return hipSuccess;
    size_t n16 = bytes / 16, ntail = bytes % 16;
    size_t blocks = (n16 + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, s, (uint4 *)p, n16,
                       (unsigned char *)p + n16 * 16, ntail);
    return hipGetLastError();
}

// Streaming device copy (measurement helper: the achievable HBM rate of a
// plain read + write, to set the other kernels' traffic against).  Each
// thread moves four 16-byte units per round, all loads issued before the
// stores; a grid of a few workgroups per compute unit strides over the
// buffer.  A tail below 64 bytes is copied byte by byte by block 0.
__global__ __launch_bounds__(256) void k_copy(const uint4 *__restrict__ src, uint4 *__restrict__ dst, size_t n16,
                                              const unsigned char *__restrict__ stail,
                                              unsigned char *__restrict__ dtail, size_t ntail)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n16; i += 4 * stride) {
        uint4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
        dst[i] = a;
        dst[i + stride] = b;
        dst[i + 2 * stride] = c;
        dst[i + 3 * stride] = d;
    }
    for (; i < n16; i += stride) dst[i] = src[i];
    if (blockIdx.x == 0)
        for (size_t t = threadIdx.x; t < ntail; t += blockDim.x) dtail[t] = stail[t];
}

hipError_t launch_copy(void *dst, const void *src, size_t bytes, int cus, hipStream_t s)
{
    if (bytes == 0) return hipSuccess;
    const size_t n16 = bytes / 16, ntail = bytes % 16;
    size_t blocks = (n16 + 255) / 256;
    const size_t cap = (size_t)(cus > 0 ? cus : 256) * 8;
    if (blocks > cap) blocks = cap;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, s, (const uint4 *)src, (uint4 *)dst, n16,
                       (const unsigned char *)src + n16 * 16, (unsigned char *)dst + n16 * 16, ntail);
    return hipGetLastError();
}

// Native two-component vector of a real type (one memory operation per
// complex value).
template <typename R> struct Cplx;
template <> struct Cplx<float> { typedef float T __attribute__((ext_vector_type(2))); };
template <> struct Cplx<double> { typedef double T __attribute__((ext_vector_type(2))); };

// Values in sorted order for the spread: fs[i] = f[perm[i]] (dense stores;
// the reads gather from f).
template <typename R>
__global__ void k_gather(const R *__restrict__ f, const int *__restrict__ perm, long long total,
                         R *__restrict__ fs)
{
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    // one complex value: a single 8- or 16-byte load and store
    using C = typename Cplx<R>::T;
    reinterpret_cast<C *>(fs)[i] = reinterpret_cast<const C *>(f)[perm[i]];
}

// Interpolation outputs back to the caller's order: f[j] = outs[ipos[j]],
// ipos[j] = sorted position of point j (dense stores).
template <typename R>
__global__ void k_scatter(const R *__restrict__ outs, const int *__restrict__ ipos, long long total,
                          R *__restrict__ f)
{
    long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= total) return;
    using C = typename Cplx<R>::T;
    reinterpret_cast<C *>(f)[j] = reinterpret_cast<const C *>(outs)[ipos[j]];
}

// outs4 per sorted point: p, d0 p, d1 p, d2 p (complex).  grad_x = Re(f conj(d p)).
template <typename R>
// grad_x has d = 3 - flat columns: the derivatives along the flat leading
// dims (which carry no coordinate) are not returned.
__global__ void k_grad_finish(const R *__restrict__ outs4, const R *__restrict__ f,
                              const int *__restrict__ ipos, long long total, int flat, R *__restrict__ grad_f,
                              R *__restrict__ grad_x)
{
    long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= total) return;
    const R *o = outs4 + (long long)ipos[j] * 8;
    if (grad_f) {
        grad_f[2 * j] = o[0];
        grad_f[2 * j + 1] = o[1];
    }
    if (grad_x) {
        const int d = 3 - flat;
        R fr = f[2 * j], fi = f[2 * j + 1];
        for (int t = flat; t < 3; ++t) grad_x[d * j + (t - flat)] = fr * o[2 + 2 * t] + fi * o[3 + 2 * t];
    }
}

template <typename R>
hipError_t launch_gather(const void *f, const int *perm, long long total, R *fs, hipStream_t s)
{
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather<R>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, (const R *)f, perm,
                       total, fs);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_scatter(const R *outs, const int *ipos, long long total, void *f, hipStream_t s)
{
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scatter<R>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, outs, ipos,
                       total, (R *)f);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_grad_finish(const R *outs4, const void *f, const int *ipos, long long total, int flat,
                              void *grad_f, void *grad_x, hipStream_t s)
{
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_grad_finish<R>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, outs4,
                       (const R *)f, ipos, total, flat, (R *)grad_f, (R *)grad_x);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Eq. (12) reciprocal sum.  One thread per k in I_N; k = 0 excluded.
constexpr int kEwThreads = 256;

template <typename R>
__global__ __launch_bounds__(kEwThreads) void k_ewald(const R *__restrict__ S, int N0, int N1, int N2,
                                                      double L, double alpha, double *__restrict__ part,
                                                      R *__restrict__ gbar)
{
    __shared__ double sh[kEwThreads];
    long long tot = (long long)N0 * N1 * N2;
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double e = 0.0;
    if (i < tot) {
        long long k0 = i / ((long long)N1 * N2) - N0 / 2;
        long long k1 = (i / N2) % N1 - N1 / 2;
        long long k2 = i % N2 - N2 / 2;
        double k2s = (double)(k0 * k0 + k1 * k1 + k2 * k2);
        double w = 0.0;
        if (k2s > 0.0) w = exp(-M_PI * M_PI * k2s / (alpha * L * alpha * L)) / k2s;
        double sr = (double)S[2 * i], si = (double)S[2 * i + 1];
        e = w * (sr * sr + si * si) / (2.0 * M_PI * L);
        if (gbar) {
            // d/dRe S + i d/dIm S of w |S|^2 / (2 pi L)
            gbar[2 * i] = (R)(w * sr / (M_PI * L));
            gbar[2 * i + 1] = (R)(w * si / (M_PI * L));
        }
    }
    sh[threadIdx.x] = e;
    __syncthreads();
    for (int off = kEwThreads / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// Fixed-order final sum of the block partials (deterministic).
__global__ __launch_bounds__(kEwThreads) void k_sum_partials(const double *__restrict__ part, int n,
                                                             double *__restrict__ out)
{
    __shared__ double sh[kEwThreads];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += part[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int off = kEwThreads / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

hipError_t launch_sum_partials(const double *part, int n, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kEwThreads), 0, s, part, n, out);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_ewald(const void *S, const Xform &X, double L, double alpha, double *partials,
                        int nblocks, double *energy, void *gbar, hipStream_t s)
{
    hipLaunchKernelGGL(k_ewald<R>, dim3(nblocks), dim3(kEwThreads), 0, s, (const R *)S, X.N[0], X.N[1],
                       X.N[2], L, alpha, partials, (R *)gbar);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kEwThreads), 0, s, partials, nblocks, energy);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Eq. (11) real-space Ewald sum by direct pairs under the minimum-image
// convention (valid when erfc(alpha r) is negligible beyond half the box):
//   U = 1/2 sum_i sum_{j != i} q_i q_j erfc(alpha r_ij) / r_ij   (r_ij < rcut)
//   F_i = sum_j q_i q_j [erfc(alpha r)/r + 2 alpha/sqrt(pi) exp(-alpha^2 r^2)] d_ij / r^2
// One thread per ion i; the j loop streams through LDS tiles of 256 ions.
constexpr int kRealTile = kEwaldRealTile;

__global__ __launch_bounds__(kRealTile) void k_ewald_real(const double *__restrict__ r,
                                                          const double *__restrict__ q, long long M,
                                                          double L, double alpha, double rcut2,
                                                          double *__restrict__ part,
                                                          double *__restrict__ forces)
{
    __shared__ double sx[kRealTile], sy[kRealTile], sz[kRealTile], sq[kRealTile];
    __shared__ double red[kRealTile];
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < M;
    const double xi = valid ? r[3 * i] : 0.0, yi = valid ? r[3 * i + 1] : 0.0, zi = valid ? r[3 * i + 2] : 0.0;
    const double qi = valid ? q[i] : 0.0;
    const double c2 = 2.0 * alpha / sqrt(M_PI), invL = 1.0 / L;
    double e = 0.0, fx = 0.0, fy = 0.0, fz = 0.0;
    for (long long j0 = 0; j0 < M; j0 += kRealTile) {
        long long j = j0 + threadIdx.x;
        __syncthreads();
        sx[threadIdx.x] = j < M ? r[3 * j] : 0.0;
        sy[threadIdx.x] = j < M ? r[3 * j + 1] : 0.0;
        sz[threadIdx.x] = j < M ? r[3 * j + 2] : 0.0;
        sq[threadIdx.x] = j < M ? q[j] : 0.0;
        __syncthreads();
        const int nj = (int)min((long long)kRealTile, M - j0);
        for (int t = 0; t < nj; ++t) {
            if (j0 + t == i) continue;
            double dx = xi - sx[t], dy = yi - sy[t], dz = zi - sz[t];
            dx -= L * rint(dx * invL);
            dy -= L * rint(dy * invL);
            dz -= L * rint(dz * invL);
            double d2 = dx * dx + dy * dy + dz * dz;
            if (d2 >= rcut2) continue;
            double d = sqrt(d2);
            double qq = qi * sq[t];
            double ec = erfc(alpha * d) / d;
            e += 0.5 * qq * ec;
            double g = qq * (ec + c2 * exp(-alpha * alpha * d2)) / d2;
            fx += g * dx;
            fy += g * dy;
            fz += g * dz;
        }
    }
    if (valid && forces) {
        forces[3 * i] = fx;
        forces[3 * i + 1] = fy;
        forces[3 * i + 2] = fz;
    }
    red[threadIdx.x] = e;
    __syncthreads();
    for (int off = kRealTile / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

hipError_t launch_ewald_real(const double *r, const double *q, long long M, double L, double alpha,
                             double rcut, double *partials, double *energy, double *forces, hipStream_t s)
{
    int nb = (int)((M + kRealTile - 1) / kRealTile);
    hipLaunchKernelGGL(k_ewald_real, dim3(nb), dim3(kRealTile), 0, s, r, q, M, L, alpha, rcut * rcut, partials,
                       forces);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kEwThreads), 0, s, partials, nb, energy);
    return hipGetLastError();
}

#define HPNFFT_INST(R)                                                                             \
    template hipError_t launch_gather<R>(const void *, const int *, long long, R *, hipStream_t);   \
    template hipError_t launch_scatter<R>(const R *, const int *, long long, void *, hipStream_t); \
    template hipError_t launch_grad_finish<R>(const R *, const void *, const int *, long long, int,\
                                              void *, void *, hipStream_t);                        \
    template hipError_t launch_ewald<R>(const void *, const Xform &, double, double, double *, int, \
                                        double *, void *, hipStream_t);
HPNFFT_INST(double)
HPNFFT_INST(float)
#undef HPNFFT_INST

}  // namespace hpnfft
