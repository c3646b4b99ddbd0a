// FFT passes over the oversampled grid (Section 2: the FFT step of the
// gridding scheme; Algorithm 2 runs a forward FFT, Algorithm 5 an inverse one)
// with the crop to I_N and the division by the window's Fourier coefficients
// ("Scaling"; "Subdividing" on the way back) fused into the first / last pass.
//
// One pass transforms all pencils along one dimension.  A workgroup loads
// `count` pencils (coalesced: a run of contiguous elements per pencil row),
// runs a mixed-radix (8, 4, 2, 3, 5, 7) Stockham autosort FFT in LDS with FP64
// twiddles (rounded once for the float path), and stores only the outputs the
// next step needs.  The stages run in place in one LDS buffer (each thread
// reads its butterflies' inputs into registers before any output is
// written), so more workgroups fit on a compute unit.  The passes are HBM-bound; pruning keeps the traffic at
// about 2.6 grid volumes per transform instead of 6.
//
// Adjoint (sign -):  grid[n0][n1][n2] --dim2--> A[n0][n1][N2] --dim1--> B[n0][N1][N2]
//                    --dim0, x 1/c_k--> fhat[N0][N1][N2]
// Forward (sign +):  fhat --x 1/c_k, pad, dim0--> B --dim1--> A --dim2--> grid
// Frequency k of a length-n transform sits at bin k mod n; the cropped
// (centred) arrays store k at k + N/2.
#include <algorithm>

#include "internal.h"

namespace hpnfft {

constexpr int kFftThreads = 256;
constexpr int kFftCap = 2048;  // complex elements per LDS buffer (count * n)
constexpr int kLoadU = 8;      // loads in flight per thread: kLoadU * kFftThreads >= kFftCap

template <typename R> struct C2 { R x, y; };
// loads and stores through global pointers, member by member (the compiler
// merges them into one 8- or 16-byte access)
template <typename R> __device__ inline C2<R> gload(gptr<const C2<R>> p) { return C2<R>{p->x, p->y}; }
template <typename R> __device__ inline void gstore(gptr<C2<R>> p, C2<R> v)
{
    p->x = v.x;
    p->y = v.y;
}

template <typename R> __device__ inline C2<R> cmul(C2<R> a, C2<R> b)
{
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename R> __device__ inline C2<R> cadd(C2<R> a, C2<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R> __device__ inline C2<R> csub(C2<R> a, C2<R> b) { return {a.x - b.x, a.y - b.y}; }
// multiply by i*S (S = +1 or -1)
template <int S, typename R> __device__ inline C2<R> mul_is(C2<R> a) { return {-S * a.y, S * a.x}; }

// In-register DFT of length RAD with kernel exp(S 2 pi i n k / RAD).
template <int S, typename R> __device__ inline void dft2(C2<R> *v)
{
    C2<R> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}
template <int S, typename R> __device__ inline void dft4(C2<R> *v)
{
    C2<R> a0 = v[0], a1 = v[1], a2 = v[2], a3 = v[3];
    C2<R> s02 = cadd(a0, a2), d02 = csub(a0, a2);
    C2<R> s13 = cadd(a1, a3), d13 = mul_is<S>(csub(a1, a3));
    v[0] = cadd(s02, s13);
    v[2] = csub(s02, s13);
    v[1] = cadd(d02, d13);
    v[3] = csub(d02, d13);
}
template <int S, typename R> __device__ inline void dft8(C2<R> *v)
{
    C2<R> e[4] = {v[0], v[2], v[4], v[6]};
    C2<R> o[4] = {v[1], v[3], v[5], v[7]};
    dft4<S>(e);
    dft4<S>(o);
    const R h = (R)0.70710678118654752440;
    // w^k = exp(S 2 pi i k / 8)
    C2<R> w1 = {h, S * h}, w3 = {-h, S * h};
    C2<R> t0 = o[0], t1 = cmul(o[1], w1), t2 = mul_is<S>(o[2]), t3 = cmul(o[3], w3);
    v[0] = cadd(e[0], t0);
    v[4] = csub(e[0], t0);
    v[1] = cadd(e[1], t1);
    v[5] = csub(e[1], t1);
    v[2] = cadd(e[2], t2);
    v[6] = csub(e[2], t2);
    v[3] = cadd(e[3], t3);
    v[7] = csub(e[3], t3);
}
template <int S, typename R> __device__ inline void dft3(C2<R> *v)
{
    const R c = (R)0.86602540378443864676;  // sqrt(3)/2
    C2<R> t1 = cadd(v[1], v[2]), t2 = csub(v[1], v[2]);
    C2<R> a = {v[0].x - (R)0.5 * t1.x, v[0].y - (R)0.5 * t1.y};
    C2<R> b = {-S * c * t2.y, S * c * t2.x};  // i S (sqrt3/2) t2
    v[0] = cadd(v[0], t1);
    v[1] = cadd(a, b);
    v[2] = csub(a, b);
}

// Odd prime radix P (5 or 7) as a direct DFT: the P - 1 nontrivial outputs
// pair up as k and P - k, which share the cosine sums of v[r] + v[P - r] and
// the sine sums of v[r] - v[P - r] (cos and sin of 2 pi j / P below, j = 1 ..
// (P - 1) / 2, to 20 digits).
template <int P> struct RootsOf;
template <> struct RootsOf<5> {
    static constexpr double c[3] = {1.0, 0.30901699437494742410, -0.80901699437494742410};
    static constexpr double s[3] = {0.0, 0.95105651629515357212, 0.58778525229247312917};
};
template <> struct RootsOf<7> {
    static constexpr double c[4] = {1.0, 0.62348980185873353053, -0.22252093395631440429,
                                    -0.90096886790241912624};
    static constexpr double s[4] = {0.0, 0.78183148246802980871, 0.97492791218182360702,
                                    0.43388373911755812048};
};
template <int P, int S, typename R> __device__ inline void dft_odd(C2<R> *v)
{
    constexpr int H = (P - 1) / 2;
    C2<R> sp[H + 1], dm[H + 1];
#pragma unroll
    for (int r = 1; r <= H; ++r) {
        sp[r] = cadd(v[r], v[P - r]);
        dm[r] = csub(v[r], v[P - r]);
    }
    C2<R> out[P];
    out[0] = v[0];
#pragma unroll
    for (int r = 1; r <= H; ++r) out[0] = cadd(out[0], sp[r]);
#pragma unroll
    for (int k = 1; k <= H; ++k) {
        // exp(S 2 pi i r k / P) = cos(2 pi (rk mod P)/P) + i S sin(...)
        C2<R> a = v[0], b = {R(0), R(0)};
#pragma unroll
        for (int r = 1; r <= H; ++r) {
            int q = (r * k) % P;
            const bool neg = q > H;     // sin(2 pi q / P) = -sin(2 pi (P - q) / P)
            const int j = neg ? P - q : q;
            const R cr = (R)RootsOf<P>::c[j];
            const R sr = neg ? (R)(-RootsOf<P>::s[j]) : (R)RootsOf<P>::s[j];
            a.x += cr * sp[r].x;
            a.y += cr * sp[r].y;
            b.x += sr * dm[r].x;
            b.y += sr * dm[r].y;
        }
        // out[k] = a + i S b,  out[P - k] = a - i S b
        const C2<R> ib = mul_is<S>(b);
        out[k] = cadd(a, ib);
        out[P - k] = csub(a, ib);
    }
#pragma unroll
    for (int r = 0; r < P; ++r) v[r] = out[r];
}

// One in-place Stockham stage of radix RAD for `count` pencils of length n:
// every thread first reads the inputs of its butterflies into registers,
// then (after a barrier) writes their outputs to the same buffer, so one LDS
// buffer serves all stages.
template <int RAD, int S, typename R>
__device__ inline void stage(C2<R> *buf, const C2<R> *tw, int n, int ld, int count, int Ns)
{
    constexpr int MAXB = (kFftCap + RAD * kFftThreads - 1) / (RAD * kFftThreads);  // butterflies per thread
    const int nb = n / RAD;
    const int tstep = n / (Ns * RAD);
    const int total = count * nb;
    C2<R> v[MAXB][RAD];
    int dst[MAXB];
#pragma unroll
    for (int q = 0; q < MAXB; ++q) {
        const int t = threadIdx.x + q * kFftThreads;
        dst[q] = -1;
        if (t < total) {
            const int pen = t / nb, j = t - pen * nb;
            const int k = j % Ns;
            const C2<R> *sp = buf + pen * ld;
#pragma unroll
            for (int r = 0; r < RAD; ++r) v[q][r] = sp[j + r * nb];
            if (Ns > 1) {
#pragma unroll
                for (int r = 1; r < RAD; ++r) v[q][r] = cmul(v[q][r], tw[k * r * tstep]);
            }
            if (RAD == 2) dft2<S>(v[q]);
            if (RAD == 3) dft3<S>(v[q]);
            if (RAD == 4) dft4<S>(v[q]);
            if (RAD == 8) dft8<S>(v[q]);
            if (RAD == 5) dft_odd<5, S>(v[q]);
            if (RAD == 7) dft_odd<7, S>(v[q]);
            dst[q] = pen * ld + (j / Ns) * Ns * RAD + k;
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < MAXB; ++q) {
        if (dst[q] >= 0) {
#pragma unroll
            for (int r = 0; r < RAD; ++r) buf[dst[q] + r * Ns] = v[q][r];
        }
    }
    __syncthreads();
}

struct PassGeom {
    int dim, n, N, Lin, Lout, inner;
    long long outer_len;  // number of outer indices
    bool crop;            // adjoint: keep N of n outputs
    bool roll_out, roll_in;
};

__device__ inline PassGeom pass_geom(int pass, const Xform &X)
{
    PassGeom g;
    switch (pass) {
    case P_ADJ0: g.dim = 2; g.inner = 1; g.outer_len = (long long)X.n[0] * X.n[1]; break;
    case P_ADJ1: g.dim = 1; g.inner = X.N[2]; g.outer_len = X.n[0]; break;
    case P_ADJ2: g.dim = 0; g.inner = X.N[1] * X.N[2]; g.outer_len = 1; break;
    case P_FWD0: g.dim = 0; g.inner = X.N[1] * X.N[2]; g.outer_len = 1; break;
    case P_FWD1: g.dim = 1; g.inner = X.N[2]; g.outer_len = X.n[0]; break;
    default:     g.dim = 2; g.inner = 1; g.outer_len = (long long)X.n[0] * X.n[1]; break;
    }
    g.n = X.n[g.dim];
    g.N = X.N[g.dim];
    g.crop = pass <= P_ADJ2;
    g.Lin = g.crop ? g.n : g.N;
    g.Lout = g.crop ? g.N : g.n;
    g.roll_out = pass == P_ADJ2;
    g.roll_in = pass == P_FWD0;
    return g;
}

// Source and destination arrays of a pass.
template <typename R> struct PassArrays {
    gptr<const C2<R>> src;
    gptr<C2<R>> dst;
};
template <typename R> __device__ inline PassArrays<R> pass_arrays(int pass, const Xform &X, void *fhat_base)
{
    PassArrays<R> a;
    gptr<C2<R>> fh = as_global(reinterpret_cast<C2<R> *>(fhat_base)) + X.foff;
    switch (pass) {
    case P_ADJ0: a.src = as_global((const C2<R> *)X.grid); a.dst = as_global((C2<R> *)X.tmpA); break;
    case P_ADJ1: a.src = as_global((const C2<R> *)X.tmpA); a.dst = as_global((C2<R> *)X.tmpB); break;
    case P_ADJ2: a.src = as_global((const C2<R> *)X.tmpB); a.dst = fh; break;
    case P_FWD0: a.src = fh; a.dst = as_global((C2<R> *)X.tmpB); break;
    case P_FWD1: a.src = as_global((const C2<R> *)X.tmpB); a.dst = as_global((C2<R> *)X.tmpA); break;
    default:     a.src = as_global((const C2<R> *)X.tmpA); a.dst = as_global((C2<R> *)X.grid); break;
    }
    return a;
}

// element (pencil p, position j) of an array with L positions per pencil
__device__ inline long long pass_addr(const FItem &W, int inner, int p, int j, int L)
{
    if (inner == 1) return ((long long)W.outer + p) * L + j;
    return ((long long)W.outer * L + j) * inner + W.inner0 + p;
}

// One item's input, in registers: kLoadU values per thread and their LDS
// positions (-1: none).  Crop passes load all n positions of each pencil;
// pad passes load the N nonzero ones (with the roll-off factors of the
// Subdividing step in the first forward pass) into their FFT bins.
template <typename R> struct PassLoad {
    R vx[kLoadU], vy[kLoadU];
    int at[kLoadU];
};
template <typename R>
__device__ inline void pass_issue(int pass, const Xform &X, const FItem &W, void *fhat_base, PassLoad<R> &L)
{
    const PassGeom g = pass_geom(pass, X);
    const PassArrays<R> a = pass_arrays<R>(pass, X, fhat_base);
    const int n = g.n, ld = n, cnt = W.count, inner = g.inner;
    const int Lin = g.crop ? n : g.N;
    const int tot = cnt * Lin;
    const int tid = threadIdx.x, nthr = blockDim.x;
#pragma unroll
    for (int u = 0; u < kLoadU; ++u) {
        const int e = tid + u * nthr;
        const int ec = e < tot ? e : tot - 1;  // clamped: no branch around the load
        int p, j;
        if (inner == 1) {
            p = ec / Lin;
            j = ec - p * Lin;
        } else {
            j = ec / cnt;
            p = ec - j * cnt;
        }
        C2<R> w = gload<R>(a.src + pass_addr(W, inner, p, j, Lin));
        if (!g.crop) {
            if (g.roll_in) {
                const int ii = W.inner0 + p;
                const double f = as_global(X.roll[0])[j] * as_global(X.roll[1])[ii / X.N[2]] *
                                 as_global(X.roll[2])[ii % X.N[2]];
                w.x = (R)(w.x * f);
                w.y = (R)(w.y * f);
            }
            int bin = j - g.N / 2;
            if (bin < 0) bin += n;
            j = bin;
        }
        L.vx[u] = w.x;
        L.vy[u] = w.y;
        L.at[u] = e < tot ? p * ld + j : -1;
    }
}

// ODD: grids with factors 5 or 7 (their stages hold more values per thread;
// the other grids run a variant without them, with fewer registers).
template <typename R, int S, bool ODD>
__global__ __launch_bounds__(kFftThreads) void k_fft(int pass, const Xform *__restrict__ xfs,
                                                     const FItem *__restrict__ items, int nitems, void *fhat_base)
{
    extern __shared__ __align__(16) unsigned char smem[];
    C2<R> *buf = reinterpret_cast<C2<R> *>(smem);
    C2<R> *tw = buf + kFftCap;
    const int tid = threadIdx.x, nthr = blockDim.x;
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const FItem W = items[it];
        const Xform &X = xfs[W.xf];
        const PassGeom g = pass_geom(pass, X);
        const int n = g.n, ld = n, cnt = W.count;
        // all of the item's loads are issued before any LDS write
        PassLoad<R> ld_regs;
        pass_issue<R>(pass, X, W, fhat_base, ld_regs);
        // twiddles exp(S 2 pi i j / n) of this dimension (the table holds
        // exp(-2 pi i j / n))
        const gptr<const C2<R>> twg = as_global(reinterpret_cast<const C2<R> *>(X.tw[g.dim]));
        for (int j = tid; j < n; j += nthr) {
            C2<R> w = gload<R>(twg + j);
            if (S > 0) w.y = -w.y;
            tw[j] = w;
        }
        // pad passes: the positions no input lands on are zero
        if (!g.crop) {
            const int z0 = g.N - g.N / 2, z1 = n - g.N / 2;  // [z0, z1) holds no data
            const int zw = z1 - z0;
            for (int e = tid; e < cnt * zw; e += nthr) {
                const int p = e / zw, j = z0 + (e - p * zw);
                buf[p * ld + j] = C2<R>{R(0), R(0)};
            }
        }
#pragma unroll
        for (int u = 0; u < kLoadU; ++u)
            if (ld_regs.at[u] >= 0) buf[ld_regs.at[u]] = C2<R>{ld_regs.vx[u], ld_regs.vy[u]};
        __syncthreads();

        // ---- Stockham stages: radix 8 first, then 4, 2, 3, 5, 7 ----
        int rem = n, Ns = 1;
        while (rem > 1) {
            const int rad = (rem % 8 == 0) ? 8 : (rem % 4 == 0) ? 4 : (rem % 2 == 0) ? 2 : (rem % 3 == 0) ? 3
                          : (rem % 5 == 0) ? 5 : 7;
            switch (rad) {
            case 8: stage<8, S, R>(buf, tw, n, ld, cnt, Ns); break;
            case 4: stage<4, S, R>(buf, tw, n, ld, cnt, Ns); break;
            case 2: stage<2, S, R>(buf, tw, n, ld, cnt, Ns); break;
            case 3: stage<3, S, R>(buf, tw, n, ld, cnt, Ns); break;
            default:
                if constexpr (ODD) {
                    if (rad == 5) stage<5, S, R>(buf, tw, n, ld, cnt, Ns);
                    else stage<7, S, R>(buf, tw, n, ld, cnt, Ns);
                }
                break;
            }
            Ns *= rad;
            rem /= rad;
        }

        // ---- store (crop to I_N and Scaling in the last adjoint pass) ----
        const PassArrays<R> a = pass_arrays<R>(pass, X, fhat_base);
        const gptr<const double> roll0 = as_global(X.roll[0]), roll1 = as_global(X.roll[1]),
                                 roll2 = as_global(X.roll[2]);
        const int Lout = g.Lout, tot = cnt * Lout, inner = g.inner;
        for (int e = tid; e < tot; e += nthr) {
            int p, o;
            if (inner == 1) { p = e / Lout; o = e - p * Lout; }
            else { o = e / cnt; p = e - o * cnt; }
            int bin = o;
            if (g.crop) {
                bin = o - g.N / 2;
                if (bin < 0) bin += n;
            }
            C2<R> v = buf[p * ld + bin];
            if (g.roll_out) {
                const int ii = W.inner0 + p;
                const double f = roll0[o] * roll1[ii / X.N[2]] * roll2[ii % X.N[2]];
                v.x = (R)(v.x * f);
                v.y = (R)(v.y * f);
            }
            gstore<R>(a.dst + pass_addr(W, inner, p, o, Lout), v);
        }
        __syncthreads();  // the next item writes the buffer
    }
}

template <typename R>
hipError_t launch_fft(int pass, const Xform *dxf, const FItem *items, int nitems, int max_n, bool odd,
                      void *fhat_base, hipStream_t s)
{
    if (nitems <= 0) return hipSuccess;
    const size_t lds = (size_t)(kFftCap + max_n) * 2 * sizeof(R);
    const bool adj = pass <= P_ADJ2;
    auto kern = adj ? (odd ? k_fft<R, -1, true> : k_fft<R, -1, false>)
                    : (odd ? k_fft<R, 1, true> : k_fft<R, 1, false>);
    hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
    }
    // one workgroup per item up to a few rounds of the chip (LDS, 8 x 256
    // threads per CU); beyond that workgroups take several items in turn
    const int per_cu = std::max(1, std::min(8, (int)((160 * 1024) / (lds + 512))));
    const int grid = std::min(nitems, cus * per_cu * 4);
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kFftThreads), lds, s, pass, dxf, items, nitems, fhat_base);
    return hipGetLastError();
}

template hipError_t launch_fft<double>(int, const Xform *, const FItem *, int, int, bool, void *, hipStream_t);
template hipError_t launch_fft<float>(int, const Xform *, const FItem *, int, int, bool, void *, hipStream_t);

}  // namespace hpnfft
