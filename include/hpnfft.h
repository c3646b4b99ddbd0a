/*
 * hpnfft — nonequispaced fast Fourier transform on AMD MI355X (gfx950).
 *
 * C-ABI of the library.  Plain pointers and sizes only; nothing throws across
 * this boundary.  Every call returns HPNFFT_OK (0) or a negative status code.
 *
 * What is computed (Yang & Wang, arXiv 2001.01583, Section 1):
 *   frequency box  I_N = { k in Z^d : -N_t/2 <= k_t < N_t/2 },
 *   points x_j in [-1/2, 1/2)^d, j = 0 .. M-1,
 *   adjoint  (the paper's NDFT, Eq. (5)):     fhat(k) = sum_j f_j e^{-2 pi i k.x_j}
 *   forward  (the paper's "inverse", Eq. (6)): f_j = sum_{k in I_N} fhat(k) e^{+2 pi i k.x_j}
 * Eq. (6) is the conjugate transpose A^H of the matrix A of Eq. (5), not an
 * inverse (Section 1, the matrix form).  Both are evaluated approximately by
 * the gridding scheme of Section 2: window spreading onto an oversampled grid
 * of n_t = sigma * N_t cells, an FFT, and a division by the window's Fourier
 * coefficients restricted to I_N ("scaling"); the transpose runs the same
 * steps in reverse with interpolation in place of spreading.
 *
 * Layouts (all device memory, owned by the caller):
 *   x      M x d float64 (or float32 for *_f32), row-major, each in [-1/2, 1/2)
 *   f      M complex, interleaved (re, im); double for HPNFFT_F64 plans,
 *          float for HPNFFT_F32 plans
 *   fhat   prod(N) complex, C order (last dimension fastest), frequency k_t
 *          stored at index k_t + N_t/2
 * Streams: all transform calls are asynchronous on the plan's HIP stream.
 * A plan serves one call at a time: its workspace (the grid, the sorted
 * values, the outputs) and the work-queue counters of its sweep kernels
 * (which reset themselves at the end of each launch) assume that its
 * launches run in stream order.  Calls on one plan from two streams, or the
 * replay of its captured graph overlapping an eager call on another stream,
 * race; use one plan per concurrent stream.
 * The library never allocates device memory: the caller provides one
 * workspace buffer of hpnfft_workspace_size() bytes.  The only allocation
 * is 64 bytes of pinned host memory per plan (at its first set_points), the
 * target of set_points' status readback.
 */
#ifndef HPNFFT_H
#define HPNFFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define HPNFFT_OK        0
#define HPNFFT_EINVAL   (-1)  /* invalid argument (sizes, null pointer, unsupported) */
#define HPNFFT_EDOMAIN  (-2)  /* a point lies outside [-1/2,1/2)^d or is not finite */
#define HPNFFT_ENOMEM   (-3)  /* host allocation failed or workspace too small       */
#define HPNFFT_EHIP     (-4)  /* a HIP runtime call failed                           */
#define HPNFFT_ESTATE   (-5)  /* call out of order (e.g. transform before set_points)*/
#define HPNFFT_ESIZE    (-6)  /* input exceeds a fixed capacity of the library       */

/* ---- window (Section 2: a window well localised in space and frequency;
 * Section 4 compares these four).  In grid units t = n x - l, each
 * normalised to phi(0) = 1 and truncated to |t| <= m, with the Scaling
 * step's divisor D(k) = its Fourier transform at k/n cycles per cell
 * (NFFT literature: Potts, Steidl, Tasche 2001; Keiner, Kunis, Potts 2009):
 *   KAISER_BESSEL  sinh(b r)/r, r = sqrt(m^2 - t^2), b = pi (2 - 1/sigma);
 *                  D ~ I0(m sqrt(b^2 - (2 pi k/n)^2))
 *   GAUSSIAN       exp(-t^2/g), g = 2 sigma m / ((2 sigma - 1) pi);
 *                  D = sqrt(pi g) exp(-g (pi k/n)^2)
 *   BSPLINE        centred cardinal B-spline of order 2m;  D ~ sinc(pi k/n)^2m
 *   SINC_POWER     sinc(beta t)^2m, beta = pi (2 sigma - 1)/(2 m sigma);
 *                  D = (pi/beta) M_2m(pi k/(n beta)), M_2m the B-spline */
#define HPNFFT_KAISER_BESSEL 0
#define HPNFFT_GAUSSIAN      1
#define HPNFFT_BSPLINE       2
#define HPNFFT_SINC_POWER    3

/* ---- arithmetic precision of the transform -------------------------- */
#define HPNFFT_F64 0          /* complex128 values, FP64 grid, FFT and sums     */
#define HPNFFT_F32 1          /* complex64 values, FP32 grid, FFT and sums      */

/* ---- plan flags ------------------------------------------------------ */
#define HPNFFT_WITH_GRADIENT 1u  /* also tabulate window derivatives at set_points,
                                    enabling hpnfft_adjoint_backward            */
#define HPNFFT_DETERMINISTIC 2u  /* bitwise reproducible results: points sorted
                                    stably by bin and input index, every sum
                                    taken in a fixed order (one wavefront per
                                    output box in the spread, per point in the
                                    interpolation), no floating-point atomics.
                                    Repeated calls, and repeated set_points of
                                    the same points, give identical bits for a
                                    given plan and tiling.  Uses the box bins
                                    (hpnfft_set_method: LINES is refused);
                                    slower than the default paths.           */

typedef struct hpnfft_plan_s *hpnfft_plan;
typedef struct hpnfft_plan_s *hpnfft_batch;   /* a batch is a plan over B transforms */

/* Human-readable text for a status code.  Never NULL. */
const char *hpnfft_strerror(int status);

/* Create a plan for one transform (Section 1 defines d, N, M; Section 4 uses
 * sigma = 2 and the cut-off m).
 *   d          1, 2 or 3 (Section 1 states the problem for any d).  d < 3
 *              runs the three-dimensional kernels with 3 - d leading
 *              dims that carry no coordinate (N_t = 1, unit-impulse
 *              window: exact); their grid edge is the smallest even
 *              2^a 3^b 5^c 7^d >= 2m, which multiplies the spread and
 *              interpolation work by about 2m per such dim
 *   N[d]       bandwidth, each N_t even and >= 2 (Section 1)
 *   M          number of points, >= 1
 *   sigma      oversampling factor; n_t = sigma * N_t must be an even integer
 *              of the form 2^a 3^b 5^c 7^d with 2m <= n_t <= 1024
 *   m          window cut-off: 2m grid cells per dimension, 1 <= m <= 15
 *   window     HPNFFT_KAISER_BESSEL, HPNFFT_GAUSSIAN, HPNFFT_BSPLINE or
 *              HPNFFT_SINC_POWER
 *   precision  HPNFFT_F64 or HPNFFT_F32
 *   flags      0, HPNFFT_WITH_GRADIENT and/or HPNFFT_DETERMINISTIC
 * The plan starts without a workspace and without points.
 * Errors: EINVAL on any invalid argument, ENOMEM. */
int hpnfft_plan_create(hpnfft_plan *out, int d, const int64_t *N, int64_t M,
                       double sigma, int m, int window, int precision,
                       unsigned flags);

/* Destroy a plan.  Does not free the caller's workspace.  NULL is a no-op. */
int hpnfft_plan_destroy(hpnfft_plan plan);

/* HIP stream (a hipStream_t cast to void*) for all later calls; NULL is the
 * default stream.  Must not be changed while a graph captured by
 * hpnfft_batch_capture is in use. */
int hpnfft_set_stream(hpnfft_plan plan, void *hip_stream);

/* Sweep method of the spread and the interpolation (the Spreading and
 * Interpolating steps of Section 3).  Must be called before
 * hpnfft_set_workspace; resets the tiling to the method's default.
 *   HPNFFT_METHOD_LINES  points sorted into runs along dim 0 and swept with
 *                        register windows; LDS tiles with a halo of 2m - 1
 *                        cells flushed with global atomic adds (dense
 *                        point sets)
 *   HPNFFT_METHOD_BOXES  every workgroup owns one output box (>= m cells per
 *                        edge) and takes the points of the 27 boxes around
 *                        it; the grid is written once, with plain stores
 *                        (sparse point sets)
 *   HPNFFT_METHOD_AUTO   (the default) per transform: boxes below 0.1
 *                        (float64) or 0.05 (float32) points per grid cell
 *                        (environment variable HPNFFT_BOX_DENSITY overrides),
 *                        so a batch may mix the two (its tiling then sets the
 *                        line sweeps; its box transforms use 16-cell boxes)
 * The results agree to rounding; hpnfft_get_method reports the method in use
 * (LINES, BOXES, or MIXED for a batch that uses both). */
#define HPNFFT_METHOD_AUTO  0
#define HPNFFT_METHOD_LINES 1
#define HPNFFT_METHOD_BOXES 2
#define HPNFFT_METHOD_MIXED 3   /* reported by hpnfft_get_method only */
int hpnfft_set_method(hpnfft_plan plan, int method);
int hpnfft_get_method(hpnfft_plan plan, int *method);

/* Spread/interpolation tiling: tile edge in the two fastest grid dimensions
 * (cells, 4..32), slab depth along the slowest dimension (cells, 2..64) and
 * threads per workgroup (multiple of 64, <= 1024).  Pass 0 to keep a value.
 * With the box method, tile and slab are the target box edges (>= m) in
 * dims 1, 2 and in dim 0; threads is not used (512).
 * Must be called before hpnfft_set_workspace.  EINVAL if the tile does not
 * fit the 160 KiB local data share, or if 2m = 8 and the tile edge is not a
 * multiple of 8 (those plans sort points in blocks of 8 lines).
 * With 2m = 8, a tile edge of 8 and a slab depth that is a multiple of 8
 * (the default: 8, 32), and every line-method grid's n0 a multiple of 8, the
 * spread and the interpolation run as ring sweeps (one wavefront per block
 * of 8 lines through the whole slab; environment variable HPNFFT_RING=0
 * selects the staged sweeps instead); threads is then 512 whatever is
 * passed.  With 2m = 16 and every line-method grid's n0 a multiple of 16,
 * the forward's interpolation runs by groups of lines over 64-plane slabs
 * whatever the tiling (environment variable HPNFFT_LINES=0 selects the
 * staged sweep); the spread keeps the tiling. */
int hpnfft_set_tiles(hpnfft_plan plan, int tile, int slab, int threads);
int hpnfft_get_tiles(hpnfft_plan plan, int *tile, int *slab, int *threads);

/* Bytes of device workspace this plan needs (depends on the tiling). */
int hpnfft_workspace_size(hpnfft_plan plan, size_t *bytes);

/* Attach the caller's device workspace (>= hpnfft_workspace_size bytes,
 * 256-byte aligned).  Uploads the roll-off and twiddle tables.  The buffer
 * must stay alive and untouched by the caller until the plan is destroyed or
 * another workspace is set.  ENOMEM if too small. */
int hpnfft_set_workspace(hpnfft_plan plan, void *dev_ptr, size_t bytes);

/* Set the points x (device, M x d row-major, float64).  Bins and sorts them
 * and tabulates the window values (the paper's CUNFFT evaluates the window on
 * the fly, Section 1; here it is tabulated once per point set because the
 * same points serve adjoint, forward and gradient).  The caller may free x
 * afterwards.  Waits once for the plan's stream (the calling thread polls
 * the readback of the status words, keeping one host core busy until the
 * binning kernels are done), to check the domain: returns EDOMAIN if any coordinate
 * is outside [-1/2,1/2) or not finite, and the plan then has no points.
 * ESTATE if no workspace is attached. */
int hpnfft_set_points(hpnfft_plan plan, const double *x);
/* Same, for float32 coordinates (promoted exactly to float64). */
int hpnfft_set_points_f32(hpnfft_plan plan, const float *x);

/* Adjoint transform, Eq. (5) (sign -): fhat = A f.
 * f: M complex (input), fhat: prod(N) complex (output, overwritten).
 * Steps: spread f onto the grid (Section 2, "Spreading"), FFT, divide by the
 * window's Fourier coefficients on I_N ("Scaling").  ESTATE without points. */
int hpnfft_adjoint(hpnfft_plan plan, const void *f, void *fhat);

/* Forward transform, Eq. (6) (sign +, unnormalised): f = A^H fhat.
 * Steps: divide by the window's Fourier coefficients and zero-pad to the
 * oversampled grid ("Subdividing"), inverse FFT, interpolate at the points
 * ("Interpolating").  ESTATE without points. */
int hpnfft_forward(hpnfft_plan plan, const void *fhat, void *f);

/* Backward of the adjoint for a real loss L(fhat), differentiating Eq. (5):
 *   grad_fhat = dL/dRe fhat + i dL/dIm fhat       (input, prod(N) complex)
 *   grad_f    = A^H grad_fhat                      (output, M complex)
 *   grad_x    [j*d+t] = Re( f_j * conj( d/dx_{j,t} (A^H grad_fhat)(x_j) ) )
 *                                                  (output, M x d reals of the
 *                                                   plan precision)
 * f is the adjoint's input.  Needs a plan created with HPNFFT_WITH_GRADIENT
 * (else EINVAL).  grad_f or grad_x may be NULL to skip that output. */
int hpnfft_adjoint_backward(hpnfft_plan plan, const void *f, const void *grad_fhat,
                            void *grad_f, void *grad_x);

/* Reciprocal-space Ewald sum of Eq. (12) (Section 5) from the structure
 * factor S = A q computed by hpnfft_adjoint with f = q and x = r / L:
 *   energy = 1/(2 pi L) sum_{k in I_N, k != 0} exp(-pi^2 |k|^2/(alpha L)^2)/|k|^2 |S(k)|^2
 * (self term not included), accumulated in float64 on the device, written to
 * *energy_dev (one double, device memory).  If gbar is not NULL it receives
 * dE/dRe S + i dE/dIm S (prod(N) complex, plan precision), the input of
 * hpnfft_adjoint_backward that yields forces F = -(1/L) grad_x. */
int hpnfft_ewald_recip(hpnfft_plan plan, const void *S, double L, double alpha,
                       double *energy_dev, void *gbar);

/* Real-space Ewald sum of Eq. (11) (Section 5) by direct pairs under the
 * minimum-image convention, for ions r (device, M x 3 float64, coordinates in
 * a cubic box of side L) with charges q (device, M float64):
 *   energy = 1/2 sum_{i != j, r_ij < rcut} q_i q_j erfc(alpha r_ij) / r_ij
 * written to *energy_dev (device double); forces_dev (M x 3, may be NULL)
 * receives F_i = -dE/dr_i.  Requires rcut <= L/2 (one image per pair), so
 * alpha must make erfc(alpha rcut) negligible.  scratch_dev: ceil(M/256)
 * doubles of device memory.  Asynchronous on `stream` (a hipStream_t). */
int hpnfft_ewald_real(const double *r, const double *q, int64_t M, double L, double alpha,
                      double rcut, double *energy_dev, double *forces_dev,
                      double *scratch_dev, void *stream);

/* Real-space Ewald sum of Eq. (11) with cell lists, for large ionic systems
 * (Section 5's timing runs go to 12 * 64^3 ions): same sums and outputs as
 * hpnfft_ewald_real, but over pairs closer than rcut found through nc^3
 * cells of side L/nc >= rcut (nc = floor(L/rcut), at most 512), each pair
 * with its nearest periodic image, so the cost grows as M rcut^3 instead of
 * M^2.  r: device, M x 3 float64, any real coordinates (wrapped into the box
 * of side L); q: device, M float64.  Requires L >= 3 rcut (else EINVAL; use
 * hpnfft_ewald_real) and M < 2^31.  Every force has one writer; the energy
 * is summed per cell in float64 and then in a fixed order, so results are
 * bitwise reproducible.  workspace: device memory of
 * hpnfft_ewald_real_cells_workspace() bytes, 256-byte aligned (ENOMEM if
 * smaller).  Asynchronous on `stream`. */
int hpnfft_ewald_real_cells_workspace(int64_t M, double L, double rcut, size_t *bytes);
int hpnfft_ewald_real_cells(const double *r, const double *q, int64_t M, double L, double alpha,
                            double rcut, double *energy_dev, double *forces_dev, void *workspace,
                            size_t bytes, void *stream);

/* Variant of hpnfft_ewald_real that allocates nothing and takes no scratch
 * argument, for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same computation, kernels and results as hpnfft_ewald_real; the block
 * partial sums live in a static device array of the library (512 KiB per
 * device, held until the process ends), so M is limited to
 * hpnfft_ewald_real_static_max_ions() ions: larger M returns HPNFFT_ESIZE
 * before anything is launched.  Every call on one device shares that array:
 * calls that overlap on one device (different streams, or different host
 * threads without ordering) race and give wrong energies.  Nothing needs
 * clearing between calls (each call writes every partial it reads).
 * Asynchronous on `stream`. */
int hpnfft_ewald_real_static(const double *r, const double *q, int64_t M, double L, double alpha,
                             double rcut, double *energy_dev, double *forces_dev, void *stream);
/* Largest M hpnfft_ewald_real_static accepts (16,777,216). */
int64_t hpnfft_ewald_real_static_max_ions(void);

/* Tiling autotuner: times the adjoint and the forward (for gradient plans:
 * the adjoint and the backward) for each candidate tiling on the current
 * points and keeps the fastest.  scratch_f / scratch_fhat are overwritten; give them nonzero
 * values (the spread skips the grid atomics of cells that sum to zero).
 * Needs points and a workspace at least as large as the largest candidate
 * needs (query with hpnfft_workspace_size after hpnfft_set_tiles).  Writes
 * the chosen tiling to tile/slab/threads (may be NULL).  Synchronises the
 * stream. */
int hpnfft_autotune(hpnfft_plan plan, void *scratch_f, void *scratch_fhat,
                    int *tile, int *slab, int *threads);

/* Host-side domain check (no GPU needed): x is HOST memory, M x d float64
 * row-major.  Returns EDOMAIN if any coordinate lies outside [-1/2, 1/2) or
 * is not finite (Section 1 defines the points on that half-open box), and
 * writes the first offending point's index to *first_bad (-1 if none; may be
 * NULL).  EINVAL for d outside 1..3, M < 0 or a NULL x with M > 0. */
int hpnfft_check_points(const double *x, int64_t M, int d, int64_t *first_bad);

/* Streaming device-to-device copy of `bytes` bytes on `stream` (a
 * hipStream_t), for measuring the achievable HBM rate that the transform
 * kernels are compared against.  Both pointers must be 16-byte aligned
 * (else EINVAL); the ranges must not overlap.  Asynchronous. */
int hpnfft_copy(void *dst, const void *src, size_t bytes, void *stream);

/* Oversampled grid size n (d values: the plan's own dims) and points count. */
int hpnfft_plan_info(hpnfft_plan plan, int64_t *n_out, int64_t *M_out);

/* ---- batches of independent transforms ------------------------------ */
/* B transforms sharing precision, sigma, m and window; transform b has
 * bandwidth N[3b .. 3b+2] and M[b] points.  Packed buffers concatenate the
 * per-transform arrays in order: x (sum M x 3), f (sum M complex),
 * fhat (sum prod(N_b) complex). */
int hpnfft_batch_create(hpnfft_batch *out, int B, const int64_t *N, const int64_t *M,
                        double sigma, int m, int window, int precision, unsigned flags);
/* Packed set_points / adjoint / forward for a batch: each phase of every
 * transform runs as one launch over a cross-transform work list. */
int hpnfft_batch_set_points(hpnfft_batch batch, const double *x_packed);
int hpnfft_batch_adjoint(hpnfft_batch batch, const void *f_packed, void *fhat_packed);
int hpnfft_batch_forward(hpnfft_batch batch, const void *fhat_packed, void *f_packed);
/* Record the batch adjoint on the plan's (non-default) stream into a HIP
 * graph, with the given buffers; hpnfft_batch_launch replays it. */
int hpnfft_batch_capture(hpnfft_batch batch, const void *f_packed, void *fhat_packed);
int hpnfft_batch_launch(hpnfft_batch batch);
/* Element offsets of transform b in the packed point and frequency arrays. */
int hpnfft_batch_offsets(hpnfft_batch batch, int b, int64_t *point_offset,
                         int64_t *freq_offset);

/* ---- live kernel timing ------------------------------------------------ */
/* Phases timed with HIP events recorded on the plan's stream around each
 * kernel group (the FFT phases cover one pass each). */
#define HPNFFT_PH_SET_POINTS 0   /* whole set_points: bin, sort, window tables, work list */
#define HPNFFT_PH_ZERO       1   /* clearing of grids / outputs                          */
#define HPNFFT_PH_GATHER     2   /* values into sorted point order                       */
#define HPNFFT_PH_SPREAD     3   /* Spreading (adjoint)                                  */
#define HPNFFT_PH_FFT_A0     4   /* adjoint FFT pass along dim 2 (+ crop)                */
#define HPNFFT_PH_FFT_A1     5   /* adjoint FFT pass along dim 1 (+ crop)                */
#define HPNFFT_PH_FFT_A2     6   /* adjoint FFT pass along dim 0 (+ crop, Scaling)       */
#define HPNFFT_PH_FFT_F0     7   /* forward FFT pass along dim 0 (Subdividing + pad)     */
#define HPNFFT_PH_FFT_F1     8   /* forward FFT pass along dim 1 (+ pad)                 */
#define HPNFFT_PH_FFT_F2     9   /* forward FFT pass along dim 2 (+ pad)                 */
#define HPNFFT_PH_INTERP    10   /* Interpolating (forward)                              */
#define HPNFFT_PH_SCATTER   11   /* results back to the caller's point order             */
#define HPNFFT_PH_GRAD      12   /* gradient interpolation (backward)                    */
#define HPNFFT_PH_GRAD_FIN  13   /* gradient epilogue                                    */
#define HPNFFT_NPHASES      14
/* Enable (1) or disable (0) timing; either way previous records are dropped.
 * While enabled every transform call records two events per phase. */
int hpnfft_profile(hpnfft_plan plan, int enable);
/* Time only the phases whose bit (1u << phase) is set in mask (0: off);
 * previous records are dropped.  Each timed phase costs two events per call,
 * and an event between two kernels delays the second by a few microseconds,
 * so a throughput measurement times only the phase it needs. */
int hpnfft_profile_phases(hpnfft_plan plan, unsigned mask);
/* Wait for the recorded events, add their elapsed milliseconds per phase to
 * ms[HPNFFT_NPHASES] and the number of launches to counts[HPNFFT_NPHASES]
 * (either may be NULL), then drop the records. */
int hpnfft_profile_read(hpnfft_plan plan, double *ms, int64_t *counts);
/* Short name of a phase ("spread", "fft_a0", ...); "" when out of range. */
const char *hpnfft_phase_name(int phase);

/* ---- host-only helpers (no GPU needed) ------------------------------ */
/* Window `window` (HPNFFT_KAISER_BESSEL .. HPNFFT_SINC_POWER) with cut-off
 * m (1..15) in grid units t = n x - l, normalised to phi(0) = 1 and
 * truncated to |t| <= m (see the window list above), and its derivative
 * dphi/dt, at `count` points t (host arrays).  dphi may be NULL. */
int hpnfft_window_eval(int window, int m, double sigma, int64_t count, const double *t,
                       double *phi, double *dphi);
/* Roll-off factors 1/D(k) for k = -N/2 .. N/2-1 (N values; N = 1: k = 0) of
 * one dimension with grid size n, D(k) being the Fourier transform of the
 * normalised window at k/n cycles per cell: the divisor of the Scaling step
 * (Section 2). */
int hpnfft_window_rolloff(int window, int m, double sigma, int64_t n, int64_t N, double *out);

/* A-priori bound E of the one-dimensional error of the gridding scheme with
 * window `window`, cut-off m and oversampling sigma > 1 (Section 4 compares
 * the windows' accuracy against m): every output of a one-dimensional
 * transform satisfies |approximate - exact| <= E ||input||_1 (up to
 * rounding).  Formulas from the NFFT literature's error estimates (Potts,
 * Steidl, Tasche 2001); for d dimensions the bound grows to about d E.
 * sinc-power at m = 1 has no stated bound and reports 4. */
int hpnfft_window_error_bound(int window, int m, double sigma, double *bound);

#ifdef __cplusplus
}
#endif
#endif /* HPNFFT_H */
