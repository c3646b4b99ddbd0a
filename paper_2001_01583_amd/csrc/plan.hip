// Host side of the C-ABI: validation, window tables, workspace layout, and
// the kernel sequences of set_points / adjoint / forward / backward.
//
// Section 3 of the paper runs one CUNFFT per subcell (Algorithm 2:
// copy in, spread, FFT, scale, copy out; Algorithm 5: copy in, subdivide,
// inverse FFT, interpolate, copy out).  Here the data stays in HBM: the
// caller passes device pointers and every step is a kernel on the plan's
// stream.  A plan over B transforms runs each step of all B transforms as
// one launch over a combined work list (Section 3 decomposes one transform
// into subcell transforms whose results add up, Eq. (8); independent
// transforms batch the same way).
#include <unistd.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "hpnfft.h"
#include "internal.h"
#include "window.h"

namespace hpnfft {
hipError_t launch_tile_cost(const int *cell_start, const Xform &X, int T, int Zs, int m, int *lcost,
                            unsigned long long *total, hipStream_t s);
hipError_t launch_make_items(const int *lcost, int xf, const Xform &X, int T, int m, const unsigned long long *total,
                             int cap_div, int min_cap, int max_items, SItem *items, int *nitems, int *overflow,
                             hipStream_t s);
}  // namespace hpnfft

using namespace hpnfft;

namespace {

constexpr int kFftCap = 2048;  // complex elements per FFT workgroup (count * n)
constexpr int kMinCap = 2048;

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Grid edges the FFT passes factor: 2^a 3^b 5^c 7^d.
bool is_smooth(long v)
{
    if (v < 1) return false;
    for (int p : {2, 3, 5, 7})
        while (v % p == 0) v /= p;
    return v == 1;
}

int fft_count(int n)
{
    int c = 1;
    while ((c * 2) * n <= kFftCap) c *= 2;
    return c;
}

struct Layout {
    size_t counters, setp, grids, tmpA, tmpB, cell_start, scan_tmp, rank, perm, ipos, fs, xs, rec, outs, tcost, poly,
        items, fit[3], ewald, roll, tw, xf, total;
    size_t dkeys = 0, dkeys_out = 0, dvals = 0, dvals_out = 0, dsort = 0, dsort_bytes = 0;  // deterministic sort
    size_t bitems = 0;  // box work items
    size_t rec_bytes = 0;
    std::vector<size_t> grid_off, tmpA_off, tmpB_off, key_off, tcost_off, roll_off;
    std::map<int, size_t> tw_off;
    int max_items = 0, nfit[3] = {0, 0, 0}, ew_blocks = 0;
    size_t grids_bytes = 0, outs_bytes = 0;
};

}  // namespace

struct hpnfft_plan_s {
    int B = 0, m = 0, prec = 0, window = 0;
    double sigma = 2.0;
    WindowParams wp{};
    unsigned flags = 0;
    std::vector<Xform> hx;
    std::vector<long long> keys;
    long long Mtot = 0, Ftot = 0;
    Tiling til{16, 16, 1024};
    hipStream_t stream = nullptr;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    Layout L;
    bool have_ws = false, have_points = false;
    bool poly_ok = false;  // window polynomials uploaded (else direct evaluation)
    // host tables (prepare_host_tables)
    std::vector<double> h_roll, h_poly;
    std::map<int, std::vector<unsigned char>> h_tw;
    std::vector<FItem> h_fit[3];
    int nitems = 0;
    // sweep method: requested (HPNFFT_METHOD_*) and in use; the box method's
    // static work list (one item per output box) and largest box (cells)
    int method = HPNFFT_METHOD_AUTO;
    bool boxes = false;            // every transform uses boxes (tiling = box edges)
    bool any_box = false;          // some transform uses boxes
    bool any_lines = true;         // some transform uses the line sweeps
    std::vector<char> tbox;        // per transform: box method
    int max_cells = 0;
    int nbitems = 0;               // box work items (one per output box)
    std::vector<SItem> h_box_items;
    int cus = 256;
    char arch[64] = "unknown";
    int maxn = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    // set_points' readback: pinned host words and the event that marks them
    // copied (created at the first set_points, which runs on a GPU)
    int *hres = nullptr;
    hipEvent_t res_ev = nullptr;
    // live timing
    struct Rec {
        int phase;
        hipEvent_t a, b;
    };
    unsigned prof = 0;  // phases timed (bit 1 << phase)
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;

    size_t rbytes() const { return prec == HPNFFT_F32 ? 4 : 8; }
    int M2() const { return 2 * m; }
    bool grad() const { return (flags & HPNFFT_WITH_GRADIENT) != 0; }
    bool det() const { return (flags & HPNFFT_DETERMINISTIC) != 0; }
    // some grid edge has a factor 5 or 7 (the FFT then runs its odd-radix variant)
    bool odd_fft() const
    {
        for (const Xform &X : hx)
            for (int d = 0; d < 3; ++d)
                if (X.n[d] % 5 == 0 || X.n[d] % 7 == 0) return true;
        return false;
    }
    template <typename T> T *at(size_t off) const { return reinterpret_cast<T *>(ws + off); }
};

namespace {

int hip_status(hipError_t e) { return e == hipSuccess ? HPNFFT_OK : HPNFFT_EHIP; }

// ---------------------------------------------------------------------------
// Static scratch for the entry point that allocates nothing
// (hpnfft_ewald_real_static): the block partial sums of the real-space pair
// kernel live in this file-scope device array instead of a caller buffer.
// Each device holds its own copy for the life of the process.  In host code
// `scratch` only names the symbol; its device address on the current device
// comes from hipGetSymbolAddress, looked up once per device and cached.
constexpr int kStaticScratchDoubles = 65536;   // 512 KiB per device
constexpr int kMaxDevices = 64;
static __device__ __align__(256) double scratch[kStaticScratchDoubles];

std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up at the first
// call on that device).
int static_scratch(double **out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return HPNFFT_EHIP;
    if (dev < 0 || dev >= kMaxDevices) return HPNFFT_EINVAL;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return HPNFFT_EHIP;
        g_scratch_ptr[dev] = static_cast<double *>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return HPNFFT_OK;
}

// Diagnostics on stderr when the environment variable HPNFFT_LOG is set to a
// non-empty value other than "0" (read once).
bool log_on()
{
    static int on = -1;
    if (on < 0) {
        const char *v = std::getenv("HPNFFT_LOG");
        on = (v && *v && std::strcmp(v, "0") != 0) ? 1 : 0;
    }
    return on == 1;
}
void hlog(const char *fmt, ...)
{
    if (!log_on()) return;
    va_list ap;
    va_start(ap, fmt);
    std::fputs("[hpnfft] ", stderr);
    std::vfprintf(stderr, fmt, ap);
    std::fputc('\n', stderr);
    va_end(ap);
}

// ---- persistent autotuner cache -----------------------------------------
// The file named by HPNFFT_TUNE_CACHE (none: no cache) is a small JSON
// object, one entry per line:
//   {"hpnfft_tune_cache": 1,
//    "entries": {
//     "<key>": [T, Zs, threads],
//     ...
//    }}
// The key names everything the best tiling depends on: the device
// architecture and compute-unit count, precision, cut-off, window, sigma,
// the gradient flag, and per transform the grid edges and the point count
// rounded down to a power of two (batches: a hash of that list).
constexpr int kTuneCacheVersion = 3;

const char *tune_cache_path()
{
    const char *v = std::getenv("HPNFFT_TUNE_CACHE");
    return (v && *v) ? v : nullptr;
}

std::string tune_key(const hpnfft_plan_s *p)
{
    char head[256];
    std::snprintf(head, sizeof(head), "v%d|%s|cu%d|%s|m%d|w%d|s%.6g|g%d|B%d|%s", kTuneCacheVersion, p->arch,
                  p->cus, p->prec == HPNFFT_F32 ? "f32" : "f64", p->m, p->window, p->sigma, p->grad() ? 1 : 0,
                  p->B, p->boxes ? "boxes" : (p->any_box ? "mixed" : "lines"));
    std::string list;
    for (const Xform &X : p->hx) {
        int mb = 0;
        while ((2LL << mb) <= X.M) ++mb;
        char e[96];
        std::snprintf(e, sizeof(e), "|%dx%dx%d:M2^%d", X.n[0], X.n[1], X.n[2], mb);
        list += e;
    }
    if (p->B == 1) return head + list;
    unsigned long long h = 1469598103934665603ull;  // FNV-1a
    for (unsigned char c : list) h = (h ^ c) * 1099511628211ull;
    char e[40];
    std::snprintf(e, sizeof(e), "|h%016llx", h);
    return head + std::string(e);
}

// All entries of the cache file (empty if absent or unreadable).
std::map<std::string, Tiling> tune_cache_read(const char *path)
{
    std::map<std::string, Tiling> out;
    FILE *fp = std::fopen(path, "r");
    if (!fp) return out;
    char line[1024];
    int version = -1;
    while (std::fgets(line, sizeof(line), fp)) {
        if (std::strstr(line, "\"hpnfft_tune_cache\"")) {
            const char *c = std::strchr(line, ':');
            if (c) version = std::atoi(c + 1);
            continue;
        }
        const char *q0 = std::strchr(line, '"');
        const char *q1 = q0 ? std::strchr(q0 + 1, '"') : nullptr;
        const char *br = q1 ? std::strchr(q1, '[') : nullptr;
        if (!br) continue;
        Tiling t{};
        if (std::sscanf(br, "[%d , %d , %d]", &t.T, &t.Zs, &t.threads) != 3) continue;
        out[std::string(q0 + 1, q1)] = t;
    }
    std::fclose(fp);
    if (version != kTuneCacheVersion) out.clear();
    return out;
}

bool tune_cache_get(const std::string &key, Tiling *t)
{
    const char *path = tune_cache_path();
    if (!path) return false;
    auto all = tune_cache_read(path);
    auto it = all.find(key);
    if (it == all.end()) return false;
    *t = it->second;
    return true;
}

// Adds or replaces one entry; the file is rewritten through a temporary
// file and a rename, so a concurrent reader sees the old or the new file.
void tune_cache_put(const std::string &key, const Tiling &t)
{
    const char *path = tune_cache_path();
    if (!path) return;
    auto all = tune_cache_read(path);
    all[key] = t;
    std::string tmp = std::string(path) + ".tmp" + std::to_string((long long)getpid());
    FILE *fp = std::fopen(tmp.c_str(), "w");
    if (!fp) return;
    std::fprintf(fp, "{\"hpnfft_tune_cache\": %d,\n \"entries\": {\n", kTuneCacheVersion);
    size_t i = 0;
    for (const auto &kv : all)
        std::fprintf(fp, "  \"%s\": [%d, %d, %d]%s\n", kv.first.c_str(), kv.second.T, kv.second.Zs,
                     kv.second.threads, ++i < all.size() ? "," : "");
    std::fprintf(fp, " }}\n");
    const bool ok = std::fclose(fp) == 0;
    if (ok && std::rename(tmp.c_str(), path) == 0) {
        hlog("autotune: cached %s -> T=%d Zs=%d threads=%d in %s", key.c_str(), t.T, t.Zs, t.threads, path);
    } else {
        std::remove(tmp.c_str());
    }
}
#define HCHECK(x)                                                                                  \
    do {                                                                                           \
        hipError_t e_ = (x);                                                                       \
        if (e_ != hipSuccess) return HPNFFT_EHIP;                                                  \
    } while (0)

// A captured graph holds the work-item count, grid sizes, LDS sizes and
// workspace pointers of the moment it was recorded.  Every call that re-bins
// the points or re-lays out the workspace drops it (after the stream has
// finished any replay in flight); hpnfft_batch_launch then reports ESTATE
// until the batch is captured again.
void drop_graph(hpnfft_plan_s *p)
{
    if (!p->gexec && !p->graph) return;
    // (teardown: a failure leaves nothing to undo)
    (void)hipStreamSynchronize(p->stream);
    if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->gexec = nullptr;
    p->graph = nullptr;
}

// Boxes along a dim of n cells for a target box edge Tb: edges stay >= m (a
// window then reaches only the neighbouring boxes) and <= Tb when n allows.
int box_count(int n, int Tb, int m)
{
    return std::max(1, std::min(n / m, (n + Tb - 1) / Tb));
}

// Box method along one dim of n cells, for a target box edge Tb >= m:
// point bins of about max(m, 4) cells (at least m), gbox bins per output
// box, nb boxes, and an upper bound on the box edge.
struct BoxDim {
    int nbins, gbox, nb, maxw;
};
BoxDim box_dim(int n, int Tb, int m)
{
    BoxDim b;
    const int edge = std::max(m, 4);
    b.nbins = box_count(n, edge, m);
    b.gbox = std::max(1, std::min(6, Tb / edge));  // at most 8^3 bins around a box
    b.nb = (b.nbins + b.gbox - 1) / b.gbox;
    b.maxw = b.gbox * ((n + b.nbins - 1) / b.nbins);
    return b;
}

// Largest box (cells) of the box method over the plan's transforms.
long long box_max_cells(const hpnfft_plan_s *p, Tiling t)
{
    long long best = 0;
    for (int b = 0; b < p->B; ++b) {
        if (!p->tbox[b]) continue;
        const Xform &X = p->hx[b];
        long long c = 1;
        for (int d = 0; d < 3; ++d) c *= box_dim(X.n[d], d == 0 ? t.Zs : t.T, p->m).maxw;
        best = std::max(best, c);
    }
    return best;
}

// Method in use: the box method below a density of points per grid cell
// (or when requested).  Its float64 taps are single native LDS atomic adds;
// float32 taps need a compensated compare-and-swap each (gfx950's LDS
// float32 atomic add runs at 0.33 lanes per clock per compute unit against
// 7.6 for float64 and 3.5 for the 64-bit swap), so float32 switches later.
// Measured on MI355X: at 0.5 points per cell the line sweeps are 3.5-10x
// faster; at 0.01 (the 24^3-cell Ewald lattice on a 256^3 grid) the boxes
// are 2.2x (float64) and 1.3x (float32) faster.  The 256-transform float32
// batch (0.0001 - 4 points per cell per transform) runs fastest with the
// float32 switch at 0.02 now that its dense transforms take the 2m = 8 ring
// sweeps (25.05 ms; 25.8 at 0.05, 26.0 at 0.01, 27.2 at 0.005).
constexpr double kBoxDensityF64 = 0.1;
constexpr double kBoxDensityF32 = 0.02;
// The method of every transform (a batch may mix them: sparse transforms
// take boxes, dense ones the line sweeps).
void choose_methods(hpnfft_plan_s *p)
{
    double thr = p->prec == HPNFFT_F32 ? kBoxDensityF32 : kBoxDensityF64;
    // HPNFFT_BOX_DENSITY overrides the switch-over density (read per plan)
    if (const char *v = std::getenv("HPNFFT_BOX_DENSITY")) {
        char *end = nullptr;
        const double d = std::strtod(v, &end);
        if (end != v && d >= 0.0) thr = d;
    }
    p->tbox.assign(p->B, 0);
    for (int b = 0; b < p->B; ++b) {
        const Xform &X = p->hx[b];
        bool box;
        if (p->det()) box = true;  // the deterministic kernels use the box bins
        else if (p->method == HPNFFT_METHOD_LINES) box = false;
        else if (p->method == HPNFFT_METHOD_BOXES) box = true;
        else box = (double)X.M < thr * (double)X.n[0] * X.n[1] * X.n[2];
        p->tbox[b] = box;
    }
    p->any_box = std::count(p->tbox.begin(), p->tbox.end(), 1) > 0;
    p->any_lines = std::count(p->tbox.begin(), p->tbox.end(), 0) > 0;
    p->boxes = !p->any_lines;
}

// Box edges of the box transforms: the plan's tiling when every transform
// uses boxes; in a batch that mixes methods (the tiling then belongs to the
// line sweeps), 16 cells.
Tiling box_tiling(const hpnfft_plan_s *p, Tiling t) { return p->boxes ? t : Tiling{16, 16, 512}; }

// Whether the line spread of this plan runs as the ring sweep: a 2m = 8
// plan with a ring tiling whose line-method transforms all have n0 a
// multiple of 2m (HPNFFT_RING=0 turns the ring sweep off).
bool use_ring(const hpnfft_plan_s *p, const Tiling &t)
{
    static int on = -1;
    if (on < 0) {
        const char *e = getenv("HPNFFT_RING");
        on = (e && e[0] == '0') ? 0 : 1;
    }
    if (!on || !ring_tiling(p->M2(), t.T, t.Zs)) return false;
    for (size_t b = 0; b < p->hx.size(); ++b)
        if (!p->tbox[b] && p->hx[b].n[0] % p->M2()) return false;
    return true;
}

// Whether the forward's interpolation runs by groups of single lines
// (lines.h): windows of 2m = 16 cells, every line-method transform with n0 a
// multiple of 2m (HPNFFT_LINES=0 selects the staged sweep).  Measured at N =
// 64^3, M = 2^20: float64 2.94 -> 1.34 ms, float32 1.58 -> 0.91 ms for 2m =
// 16; for 2m = 10, 12 and 14 the staged sweep stays faster (float64 0.94,
// 1.35, 2.26 ms against 1.24, 1.47, 2.33 ms): with fewer taps per point the
// per-point and per-plane costs of the line groups dominate.
bool use_lines(const hpnfft_plan_s *p)
{
    static int on = -1;
    if (on < 0) {
        const char *e = getenv("HPNFFT_LINES");
        on = (e && e[0] == '0') ? 0 : 1;
    }
    const int M2 = p->M2();
    if (!on || p->det() || M2 != 16) return false;
    for (size_t b = 0; b < p->hx.size(); ++b)
        if (!p->tbox[b] && p->hx[b].n[0] % M2) return false;
    return true;
}

bool tiling_fits(const hpnfft_plan_s *p, Tiling t)
{
    if (t.T < 4 || t.T > 32 || t.Zs < 2 || t.Zs > 64) return false;
    if (t.threads < 64 || t.threads > 1024 || t.threads % 64) return false;
    if (p->any_box) {
        // box edges (dims 1, 2: T; dim 0: Zs) of at least m cells
        const Tiling bt = box_tiling(p, t);
        if (bt.T < p->m || bt.Zs < p->m) return false;
        // the box tile in LDS beside the run lists (12 KiB of static LDS)
        if (box_max_cells(p, bt) * 16 + 12 * 1024 > (long long)kLdsLimit) return false;
        if (p->boxes) return true;
    }
    if (t.T % block_w(p->M2())) return false;  // whole blocks of lines per tile row
    bool comp = p->prec == HPNFFT_F32;
    if (!use_ring(p, t) && !lds_fit(t.T, t.Zs, p->M2(), p->rbytes(), 0, comp).cap) return false;
    if (!lds_fit(t.T, t.Zs, p->M2(), p->rbytes(), 1, false).cap) return false;
    if (p->grad() && !lds_fit(t.T, t.Zs, p->M2(), p->rbytes(), 2, false).cap) return false;
    return true;
}

// Default tiling.  Measured on MI355X at 0.5 points per grid cell: single-
// line sweeps run fastest with slabs of 16 planes and tiles whose LDS
// footprint side P = T + 2m - 1 is about 20-21 cells (float64 m = 8: T = 6);
// larger tiles cut the halo traffic but leave too little LDS for staging
// points, smaller ones re-read more halo.  Blocked sweeps (2m = 8) take one
// block of lines per tile row (T = 8); in float32 with 12-plane slabs, which
// lets two workgroups share a compute unit.  The first candidate (in order of
// distance from the target) that fits is taken.
Tiling default_tiling(const hpnfft_plan_s *p)
{
    const int M2 = p->M2();
    if (p->det()) {
        // one wavefront per box: small boxes (8 cells, or m) keep many per CU
        const int Tb = std::max(8, p->m);
        if (tiling_fits(p, Tiling{Tb, Tb, 64})) return Tiling{Tb, Tb, 64};
    }
    if (p->boxes) {
        // boxes of 16 cells per edge (16 KiB of (sum, error) or float64 pairs
        // per 1024 cells: 64 KiB, two workgroups per compute unit)
        for (int Tb : {16, 12, 8})
            if (tiling_fits(p, Tiling{Tb, Tb, 512})) return Tiling{Tb, Tb, 512};
    }
    // 2m = 8: the ring sweeps (tiles of 8 x 8 lines) with the slab depth
    // that measured fastest for spread plus interpolation at 0.5 points
    // per cell (32 planes; float32 0.215 + 0.152 ms, float64 0.303 + 0.259
    // ms at N = 64^3, M = 2^20)
    if (block_w(M2) > 1) {
        const Tiling r{kRingT, 32, 512};
        if (use_ring(p, r) && tiling_fits(p, r)) return r;
    }
    // blocked 2m = 8 sweeps: tiles of one block of lines per row fit best
    const int target = block_w(M2) > 1 ? 8 : std::max(4, 22 - M2);
    std::vector<int> Ts = {4, 6, 8, 12, 16, 24, 32};
    std::stable_sort(Ts.begin(), Ts.end(),
                     [&](int a, int b) { return std::abs(a - target) < std::abs(b - target); });
    // float32 blocked sweeps: 12-plane slabs leave room for two workgroups
    // per compute unit (see two_per_cu), measured faster than 16
    const bool two = p->prec == HPNFFT_F32 && block_w(M2) > 1;
    for (int Zs : {two ? 12 : 16, two ? 16 : 12, 8})
        for (int T : Ts) {
            Tiling t{T, Zs, 1024};
            if (tiling_fits(p, t)) return t;
        }
    for (int T : {8, 6, 4})
        for (int Zs : {8, 6, 4}) {
            Tiling t{T, Zs, 1024};
            if (tiling_fits(p, t)) return t;
        }
    return Tiling{4, 4, 256};
}

void build_layout(hpnfft_plan_s *p)
{
    Layout &L = p->L;
    L = Layout();
    const size_t C = 2 * p->rbytes();
    const int T = p->til.T, Zs = p->til.Zs;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    L.counters = take(256);
    L.setp = take(256);
    // the float64 copy of the points sits at the same offset in every layout
    // (it depends on the point count only), so a re-tiled plan keeps it
    L.xs = take((size_t)p->Mtot * 24);
    size_t gbytes = 0;
    long long maxkeys = 0, maxM = 0, pairs = 0, maxF = 0;
    p->h_box_items.clear();
    p->max_cells = 0;
    for (int b = 0; b < p->B; ++b) {
        Xform &X = p->hx[b];
        X.ntx = (X.n[2] + T - 1) / T;
        X.nty = (X.n[1] + T - 1) / T;
        X.nslab = (X.n[0] + Zs - 1) / Zs;
        p->keys[b] = (long long)X.ntx * X.nty * T * T * X.n[0] + 1;
        for (int d = 0; d < 3; ++d) X.nbox[d] = X.gbox[d] = 0;
        if (p->tbox[b]) {
            // box method: sort keys are point bins; one work item per output box
            const Tiling bt = box_tiling(p, p->til);
            long long nbins = 1, nboxes = 1, cells = 1;
            for (int d = 0; d < 3; ++d) {
                const BoxDim bd = box_dim(X.n[d], d == 0 ? bt.Zs : bt.T, p->m);
                X.nbox[d] = bd.nbins;
                X.gbox[d] = bd.gbox;
                nbins *= bd.nbins;
                nboxes *= bd.nb;
                cells *= bd.maxw;
            }
            p->keys[b] = nbins + 1;
            for (long long q = 0; q < nboxes; ++q) p->h_box_items.push_back(SItem{b, (int)q, 0, 0, 0, 0, 0, 0});
            p->max_cells = std::max(p->max_cells, (int)cells);
        }
        maxkeys = std::max(maxkeys, p->keys[b]);
        maxM = std::max(maxM, X.M);
        if (!p->tbox[b]) pairs += (long long)X.ntx * X.nty * X.nslab;
        maxF = std::max(maxF, (long long)X.N[0] * X.N[1] * X.N[2]);
    }
    // grids (contiguous, zeroed by one launch)
    L.grids = off;
    for (int b = 0; b < p->B; ++b) {
        const Xform &X = p->hx[b];
        L.grid_off.push_back(off);
        gbytes += align256((size_t)X.n[0] * X.n[1] * X.n[2] * C);
        off = align256(off + (size_t)X.n[0] * X.n[1] * X.n[2] * C);
    }
    L.grids_bytes = off - L.grids;
    L.tmpA = off;
    for (int b = 0; b < p->B; ++b) {
        const Xform &X = p->hx[b];
        L.tmpA_off.push_back(take((size_t)X.n[0] * X.n[1] * X.N[2] * C));
    }
    L.tmpB = off;
    for (int b = 0; b < p->B; ++b) {
        const Xform &X = p->hx[b];
        L.tmpB_off.push_back(take((size_t)X.n[0] * X.N[1] * X.N[2] * C));
    }
    L.cell_start = off;
    for (int b = 0; b < p->B; ++b) L.key_off.push_back(take((size_t)p->keys[b] * 4));
    long long nb = (maxkeys + 4095) / 4096;
    L.scan_tmp = take((size_t)(nb + nb / 2048 + 64) * 4);
    L.rank = take((size_t)maxM * 4);
    L.perm = take((size_t)p->Mtot * 4);
    L.ipos = take((size_t)p->Mtot * 4);
    L.fs = take((size_t)p->Mtot * C);
    L.rec_bytes = rec_size(p->M2(), p->rbytes(), p->grad());
    L.rec = take((size_t)p->Mtot * L.rec_bytes);
    L.outs_bytes = (size_t)p->Mtot * C * (p->grad() ? 4 : 1);
    L.outs = take(L.outs_bytes);
    if (p->det()) {
        L.dkeys = take((size_t)maxM * 4);
        L.dkeys_out = take((size_t)maxM * 4);
        L.dvals = take((size_t)maxM * 4);
        L.dvals_out = take((size_t)maxM * 4);
        L.dsort_bytes = det_sort_bytes(maxM);
        L.dsort = take(L.dsort_bytes);
    }
    L.tcost = off;
    for (int b = 0; b < p->B; ++b) {
        const Xform &X = p->hx[b];
        L.tcost_off.push_back(take(p->tbox[b] ? 0 : (size_t)X.ntx * X.nty * X.nslab * (T * T / block_w(p->M2())) * 4));
    }
    L.max_items = (int)std::min<long long>(pairs + (long long)p->cus * 4 + 64, 0x7fffffffLL / 64);
    L.items = take((size_t)L.max_items * sizeof(SItem));
    L.bitems = take(std::max<size_t>(1, p->h_box_items.size()) * sizeof(SItem));
    for (int d = 0; d < 3; ++d) {
        long long cnt = 0;
        for (int b = 0; b < p->B; ++b) {
            const Xform &X = p->hx[b];
            int n = X.n[d], c = fft_count(n);
            if (d == 2) cnt += ((long long)X.n[0] * X.n[1] + c - 1) / c;
            if (d == 1) cnt += (long long)X.n[0] * ((X.N[2] + c - 1) / c);
            if (d == 0) cnt += ((long long)X.N[1] * X.N[2] + c - 1) / c;
        }
        L.nfit[d] = (int)cnt;
        L.fit[d] = take((size_t)cnt * sizeof(FItem));
    }
    L.ew_blocks = (int)((maxF + 255) / 256);
    L.ewald = take((size_t)L.ew_blocks * 8 + 64);
    L.poly = take((size_t)p->M2() * kPolyMax * 8);
    L.roll = off;
    for (int b = 0; b < p->B; ++b) {
        const Xform &X = p->hx[b];
        L.roll_off.push_back(take((size_t)(X.N[0] + X.N[1] + X.N[2]) * 8));
    }
    L.tw = off;
    for (int b = 0; b < p->B; ++b)
        for (int d = 0; d < 3; ++d) {
            int n = p->hx[b].n[d];
            if (!L.tw_off.count(n)) L.tw_off[n] = take((size_t)n * C);
        }
    L.xf = take((size_t)p->B * sizeof(Xform));
    L.total = off + 256;
    (void)gbytes;
}

// Window values along one dimension as polynomials: for tap t the function
// u -> Phi(u + m - 1 - t), u in [0, 1), is interpolated at nc Chebyshev points
// of v = 2u - 1 and written in monomials of v (coef[t * nc + k] multiplies
// v^k).  The window is analytic in t, so the interpolant converges fast: 10
// coefficients reach ~1e-10 and 16-17 reach ~1e-14 of the peak.  The fit is
// checked against direct evaluation on a fine grid; false if it misses tol.
bool fit_window_poly(const WindowParams &wp, int nc, double tol, std::vector<double> &coef)
{
    const int m = wp.m, M2 = 2 * m, d = nc - 1;
    coef.assign((size_t)M2 * nc, 0.0);
    for (int t = 0; t < M2; ++t) {
        std::vector<long double> fv(nc), ch(nc), mono(nc, 0.0L), tkm1(nc, 0.0L), tk(nc, 0.0L), tn(nc);
        const long double pi = 3.141592653589793238462643383279502884L;
        for (int j = 0; j < nc; ++j) {
            const long double v = cosl(pi * (j + 0.5L) / nc);
            double ph;
            win_eval(wp, (double)((v + 1.0L) / 2.0L) + (m - 1 - t), &ph, nullptr);
            fv[j] = ph;
        }
        for (int k = 0; k < nc; ++k) {
            long double a = 0.0L;
            for (int j = 0; j < nc; ++j) a += fv[j] * cosl(pi * k * (j + 0.5L) / nc);
            ch[k] = a * 2.0L / nc;
        }
        ch[0] *= 0.5L;
        // sum_k ch[k] T_k(v) in monomials, T_{k+1} = 2 v T_k - T_{k-1}
        tkm1[0] = 1.0L;
        if (d >= 1) tk[1] = 1.0L;
        mono[0] += ch[0];
        if (d >= 1) mono[1] += ch[1];
        for (int k = 1; k < d; ++k) {
            for (int i = 0; i < nc; ++i) tn[i] = (i ? 2.0L * tk[i - 1] : 0.0L) - tkm1[i];
            for (int i = 0; i < nc; ++i) mono[i] += ch[k + 1] * tn[i];
            tkm1 = tk;
            tk = tn;
        }
        for (int i = 0; i < nc; ++i) coef[(size_t)t * nc + i] = (double)mono[i];
        for (int q = 0; q <= 256; ++q) {
            const double u = q / 256.0 * (1.0 - 1e-12);
            const double v = 2.0 * u - 1.0;
            double r = coef[(size_t)t * nc + d];
            for (int k = d - 1; k >= 0; --k) r = std::fma(r, v, coef[(size_t)t * nc + k]);
            double ph;
            win_eval(wp, u + (m - 1 - t), &ph, nullptr);
            if (std::fabs(r - ph) > tol) return false;
        }
    }
    return true;
}

// Host copies of the plan's constant tables, computed once at plan creation
// (they depend on the sizes, the window and the precision, not on the tiling
// or the workspace): roll-off factors, window polynomials, twiddles and the
// FFT passes' work items.  upload_tables only copies them, so attaching a
// workspace allocates nothing on the host.
void prepare_host_tables(hpnfft_plan_s *p)
{
    p->h_roll.clear();
    for (int b = 0; b < p->B; ++b) {
        const Xform &X = p->hx[b];
        for (int d = 0; d < 3; ++d) {
            if (d < X.flat) {  // unit impulse: the Scaling step divides by 1
                p->h_roll.push_back(1.0);
                continue;
            }
            for (int k = -X.N[d] / 2; k < X.N[d] / 2; ++k)
                p->h_roll.push_back(1.0 / window_phihat(p->wp, k, X.n[d]));
        }
    }
    // window polynomials for set_points (float32 tables: 10 coefficients;
    // float64: 17); without a good fit the tables are evaluated directly
    const bool f32 = p->prec == HPNFFT_F32;
    p->poly_ok = fit_window_poly(p->wp, f32 ? kPolyF32 : kPolyF64, f32 ? 1e-9 : 5e-14, p->h_poly);
    // twiddles exp(-2 pi i j / n), computed in FP64 (long double angle), rounded once for float
    p->h_tw.clear();
    for (int b = 0; b < p->B; ++b)
        for (int d = 0; d < 3; ++d) {
            const int n = p->hx[b].n[d];
            if (p->h_tw.count(n)) continue;
            std::vector<double> w64(2 * (size_t)n);
            for (int j = 0; j < n; ++j) {
                long double a = -2.0L * 3.141592653589793238462643383279502884L * j / n;
                w64[2 * j] = (double)cosl(a);
                w64[2 * j + 1] = (double)sinl(a);
            }
            std::vector<unsigned char> bytes;
            if (f32) {
                std::vector<float> w32(w64.begin(), w64.end());
                bytes.assign(reinterpret_cast<unsigned char *>(w32.data()),
                             reinterpret_cast<unsigned char *>(w32.data()) + w32.size() * 4);
            } else {
                bytes.assign(reinterpret_cast<unsigned char *>(w64.data()),
                             reinterpret_cast<unsigned char *>(w64.data()) + w64.size() * 8);
            }
            p->h_tw[n] = std::move(bytes);
        }
    // FFT work items: `count` pencils per workgroup
    for (int d = 0; d < 3; ++d) {
        std::vector<FItem> &it = p->h_fit[d];
        it.clear();
        for (int b = 0; b < p->B; ++b) {
            const Xform &X = p->hx[b];
            int c = fft_count(X.n[d]);
            if (d == 2) {
                long long rows = (long long)X.n[0] * X.n[1];
                for (long long r = 0; r < rows; r += c)
                    it.push_back(FItem{b, (int)r, 0, (int)std::min<long long>(c, rows - r)});
            } else if (d == 1) {
                for (int o = 0; o < X.n[0]; ++o)
                    for (int i = 0; i < X.N[2]; i += c) it.push_back(FItem{b, o, i, std::min(c, X.N[2] - i)});
            } else {
                int inner = X.N[1] * X.N[2];
                for (int i = 0; i < inner; i += c) it.push_back(FItem{b, 0, i, std::min(c, inner - i)});
            }
        }
    }
}

// Point the descriptors at the workspace p->ws (host copies only).
void bind_descriptors(hpnfft_plan_s *p)
{
    const Layout &L = p->L;
    for (int b = 0; b < p->B; ++b) {
        Xform &X = p->hx[b];
        X.grid = p->ws + L.grid_off[b];
        X.tmpA = p->ws + L.tmpA_off[b];
        X.tmpB = p->ws + L.tmpB_off[b];
        double *r = p->at<double>(L.roll_off[b]);
        X.roll[0] = r;
        X.roll[1] = r + X.N[0];
        X.roll[2] = r + X.N[0] + X.N[1];
        for (int d = 0; d < 3; ++d) X.tw[d] = p->ws + L.tw_off.at(X.n[d]);
        X.key_off = (long long)((L.key_off[b] - L.cell_start) / 4);
    }
}

// Copy the tables and descriptors into the workspace p->ws.  No host or
// device allocation: the host tables were prepared at plan creation.
int upload_tables(hpnfft_plan_s *p)
{
    const Layout &L = p->L;
    bind_descriptors(p);
    size_t off = 0;
    for (int b = 0; b < p->B; ++b) {
        const Xform &X = p->hx[b];
        const size_t cnt = (size_t)X.N[0] + X.N[1] + X.N[2];
        HCHECK(hipMemcpyAsync(p->ws + L.roll_off[b], p->h_roll.data() + off, cnt * 8, hipMemcpyHostToDevice,
                              p->stream));
        off += cnt;
    }
    if (p->poly_ok)
        HCHECK(hipMemcpyAsync(p->ws + L.poly, p->h_poly.data(), p->h_poly.size() * 8, hipMemcpyHostToDevice,
                              p->stream));
    for (auto &kv : L.tw_off) {
        const std::vector<unsigned char> &t = p->h_tw.at(kv.first);
        HCHECK(hipMemcpyAsync(p->ws + kv.second, t.data(), t.size(), hipMemcpyHostToDevice, p->stream));
    }
    for (int d = 0; d < 3; ++d) {
        if ((int)p->h_fit[d].size() != L.nfit[d]) return HPNFFT_EINVAL;
        HCHECK(hipMemcpyAsync(p->ws + L.fit[d], p->h_fit[d].data(), p->h_fit[d].size() * sizeof(FItem),
                              hipMemcpyHostToDevice, p->stream));
    }
    HCHECK(hipMemcpyAsync(p->ws + L.xf, p->hx.data(), p->hx.size() * sizeof(Xform), hipMemcpyHostToDevice,
                          p->stream));
    if (p->any_box) {
        // the box method's work list does not depend on the points
        HCHECK(hipMemcpyAsync(p->ws + L.bitems, p->h_box_items.data(), p->h_box_items.size() * sizeof(SItem),
                              hipMemcpyHostToDevice, p->stream));
    }
    p->nbitems = (int)p->h_box_items.size();
    // the host sources must outlive the copies
    HCHECK(hipStreamSynchronize(p->stream));
    return HPNFFT_OK;
}

int check_plan(hpnfft_plan_s *p) { return p ? HPNFFT_OK : HPNFFT_EINVAL; }

hipEvent_t take_event(hpnfft_plan_s *p)
{
    if (!p->pool.empty()) {
        hipEvent_t e = p->pool.back();
        p->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Records an event pair around a kernel group when timing is enabled.
struct PhaseTimer {
    hpnfft_plan_s *p;
    int phase;
    hipEvent_t a = nullptr;
    PhaseTimer(hpnfft_plan_s *pl, int ph) : p(pl), phase(ph)
    {
        if (!((p->prof >> phase) & 1u)) return;
        a = take_event(p);
        if (a && hipEventRecord(a, p->stream) != hipSuccess) a = nullptr;
    }
    ~PhaseTimer()
    {
        if (!a) return;
        hipEvent_t b = take_event(p);
        if (!b) return;
        if (hipEventRecord(b, p->stream) == hipSuccess) p->recs.push_back({phase, a, b});
    }
};

void drop_records(hpnfft_plan_s *p)
{
    for (auto &r : p->recs) {
        p->pool.push_back(r.a);
        p->pool.push_back(r.b);
    }
    p->recs.clear();
}

// Bin, sort and tabulate the stored points (p->ws + L.xs); then build the
// spread / interpolation work list.  Synchronises once.
// x / x32: the caller's points (their float64 copy is written to p->ws +
// L.xs on the way), or both null to re-bin the stored copy.
int bin_points(hpnfft_plan_s *p, const double *x = nullptr, const float *x32 = nullptr)
{
    const Layout &L = p->L;
    hipStream_t s = p->stream;
    int *setp = p->at<int>(L.setp);  // [0] err, [1] nitems, [2] overflow, [4..5] total (u64)
    // the status words and the sweeps' work-queue counters (adjacent; the
    // sweeps reset their counters themselves after every launch)
    HCHECK(launch_zero(p->ws + L.counters, L.setp + 256 - L.counters, s));
    double *xs = p->at<double>(L.xs);
    const bool stored = !x && !x32;
    unsigned long long *total = reinterpret_cast<unsigned long long *>(setp + 4);
    for (int b = 0; b < p->B; ++b) {
        const Xform &X = p->hx[b];
        int *cs = p->at<int>(L.key_off[b]);
        HCHECK(launch_zero(cs, (size_t)p->keys[b] * 4, s));
        double *xb = xs + X.poff * 3;
        // the caller's points have 3 - flat coordinates each; the stored copy three
        const int dc = 3 - X.flat;
        HCHECK(launch_bin_count(stored ? xb : (x ? x + X.poff * dc : nullptr), x32 ? x32 + X.poff * dc : nullptr,
                                X.M, X, p->til.T, block_w(p->M2()), stored ? 0 : X.flat, cs, p->at<int>(L.rank),
                                setp, stored ? nullptr : xb, p->det() ? p->at<int>(L.dkeys) : nullptr, s));
        HCHECK(launch_scan(cs, p->keys[b], p->at<int>(L.scan_tmp), s));
        if (p->det()) {
            // stable order within each bin: sort (bin, input index)
            int bits = 1;
            while ((1LL << bits) < p->keys[b]) ++bits;
            HCHECK(launch_det_sort(p->at<int>(L.dkeys), X.M, bits, p->at<int>(L.dkeys_out), p->at<int>(L.dvals),
                                   p->at<int>(L.dvals_out), p->ws + L.dsort, L.dsort_bytes, X.poff,
                                   p->at<int>(L.perm), p->at<int>(L.ipos), s));
        }
        const int *fixed = p->det() ? p->at<int>(L.ipos) : nullptr;
        if (p->prec == HPNFFT_F32)
            HCHECK(launch_bin_scatter<float>(xb, nullptr, X.M, X, p->til.T, p->m, p->wp,
                                             p->poly_ok ? p->at<double>(L.poly) : nullptr, cs,
                                             p->at<int>(L.rank), p->at<int>(L.perm), p->at<int>(L.ipos),
                                             p->at<unsigned char>(L.rec), L.rec_bytes, p->grad(), fixed, s));
        else
            HCHECK(launch_bin_scatter<double>(xb, nullptr, X.M, X, p->til.T, p->m, p->wp,
                                              p->poly_ok ? p->at<double>(L.poly) : nullptr, cs,
                                              p->at<int>(L.rank), p->at<int>(L.perm), p->at<int>(L.ipos),
                                              p->at<unsigned char>(L.rec), L.rec_bytes, p->grad(), fixed, s));
        if (!p->tbox[b])
            HCHECK(launch_tile_cost(cs, X, p->til.T, p->til.Zs, p->m, p->at<int>(L.tcost_off[b]), total, s));
    }
    const int cap_div = p->cus * 4;
    for (int b = 0; b < p->B; ++b) {
        if (p->tbox[b]) continue;
        const Xform &X = p->hx[b];
        HCHECK(launch_make_items(p->at<int>(L.tcost_off[b]), b, X, p->til.T, p->m, total, cap_div, kMinCap,
                                 L.max_items, p->at<SItem>(L.items), setp + 1, setp + 2, s));
    }
    // err, nitems, overflow, pad, total cost (u64).  The copy goes to pinned
    // memory and the host polls its event: a blocking wait would leave the
    // GPU idle for the wake-up latency as well.
    if (!p->hres) {
        HCHECK(hipHostMalloc((void **)&p->hres, 64, hipHostMallocDefault));
        HCHECK(hipEventCreateWithFlags(&p->res_ev, hipEventDisableTiming));
    }
    HCHECK(hipMemcpyAsync(p->hres, setp, 6 * sizeof(int), hipMemcpyDeviceToHost, s));
    HCHECK(hipEventRecord(p->res_ev, s));
    hipError_t q;
    while ((q = hipEventQuery(p->res_ev)) == hipErrorNotReady) {
    }
    HCHECK(q);
    int host[6];
    std::memcpy(host, p->hres, sizeof(host));
    if (host[0]) return HPNFFT_EDOMAIN;
    if (host[2]) return HPNFFT_ENOMEM;
    p->nbitems = (int)p->h_box_items.size();
    p->nitems = p->any_lines ? std::min(host[1], L.max_items) : 0;
    // staging worth reserving per chunk: twice the mean points per item
    unsigned long long tot = 0;
    std::memcpy(&tot, host + 4, sizeof(tot));
    const long long mean = p->nitems > 0 ? (long long)(tot / (unsigned long long)p->nitems) : 0;
    p->til.cap_hint = (int)std::min<long long>(2 * mean + 64, 1 << 20);
    return HPNFFT_OK;
}

template <typename R> int run_adjoint(hpnfft_plan_s *p, const void *f, void *fhat)
{
    const Layout &L = p->L;
    hipStream_t s = p->stream;
    const Xform *dxf = p->at<Xform>(L.xf);
    if (p->any_lines) {  // (the box method writes every grid cell of its transforms itself)
        PhaseTimer t(p, HPNFFT_PH_ZERO);
        HCHECK(launch_zero(p->ws + L.grids, L.grids_bytes, s));
    }
    {
        PhaseTimer t(p, HPNFFT_PH_GATHER);
        HCHECK(launch_gather<R>(f, p->at<int>(L.perm), p->Mtot, p->at<R>(L.fs), s));
    }
    {
        PhaseTimer t(p, HPNFFT_PH_SPREAD);
        if (p->det())
            HCHECK(launch_spread_det<R>(p->m, dxf, p->at<SItem>(L.bitems), p->nbitems, p->max_cells,
                                        p->at<unsigned char>(L.rec), L.rec_bytes, p->at<R>(L.fs),
                                        p->at<int>(L.cell_start), s));
        else if (p->any_box)
            HCHECK(launch_spread_box<R>(p->m, dxf, p->at<SItem>(L.bitems), p->nbitems, p->at<int>(L.counters),
                                        p->max_cells, p->at<unsigned char>(L.rec), L.rec_bytes, p->at<R>(L.fs),
                                        p->at<int>(L.cell_start), s));
        if (p->any_lines) {
            Tiling t = p->til;
            t.ring = use_ring(p, t);
            HCHECK(launch_spread<R>(p->m, dxf, p->at<SItem>(L.items), p->nitems, p->at<int>(L.counters), t,
                                    p->at<unsigned char>(L.rec), L.rec_bytes, p->at<R>(L.fs),
                                    p->at<int>(L.cell_start), s));
        }
    }
    for (int pass = P_ADJ0; pass <= P_ADJ2; ++pass) {
        int d = pass == P_ADJ0 ? 2 : (pass == P_ADJ1 ? 1 : 0);
        PhaseTimer t(p, HPNFFT_PH_FFT_A0 + pass - P_ADJ0);
        HCHECK(launch_fft<R>(pass, dxf, p->at<FItem>(L.fit[d]), L.nfit[d], p->maxn, p->odd_fft(), fhat, s));
    }
    return HPNFFT_OK;
}

template <typename R> int run_to_grid(hpnfft_plan_s *p, const void *fhat)
{
    const Layout &L = p->L;
    hipStream_t s = p->stream;
    const Xform *dxf = p->at<Xform>(L.xf);
    for (int pass = P_FWD0; pass <= P_FWD2; ++pass) {
        int d = pass == P_FWD0 ? 0 : (pass == P_FWD1 ? 1 : 2);
        PhaseTimer t(p, HPNFFT_PH_FFT_F0 + pass - P_FWD0);
        HCHECK(launch_fft<R>(pass, dxf, p->at<FItem>(L.fit[d]), L.nfit[d], p->maxn, p->odd_fft(),
                             const_cast<void *>(fhat), s));
    }
    return HPNFFT_OK;
}

template <typename R> int run_forward(hpnfft_plan_s *p, const void *fhat, void *f)
{
    const Layout &L = p->L;
    hipStream_t s = p->stream;
    const Xform *dxf = p->at<Xform>(L.xf);
    // the ring interpolation stores every point's value once; the other
    // sweeps add partial sums into a cleared output
    if (p->any_box || p->det() || !use_ring(p, p->til)) {
        PhaseTimer t(p, HPNFFT_PH_ZERO);
        HCHECK(launch_zero(p->ws + L.outs, (size_t)p->Mtot * 2 * sizeof(R), s));
    }
    int rc = run_to_grid<R>(p, fhat);
    if (rc) return rc;
    {
        PhaseTimer t(p, HPNFFT_PH_INTERP);
        if (p->det())
            HCHECK(launch_interp_det<R>(p->m, false, dxf, p->B, p->Mtot, p->at<unsigned char>(L.rec), L.rec_bytes,
                                        p->at<R>(L.outs), p->cus, s));
        else if (p->any_box)
            HCHECK(launch_interp_box<R>(p->m, false, dxf, p->at<SItem>(L.bitems), p->nbitems,
                                        p->at<int>(L.counters) + 1, p->max_cells, p->at<unsigned char>(L.rec),
                                        L.rec_bytes, p->at<int>(L.cell_start), p->at<R>(L.outs), s));
        if (p->any_lines && use_lines(p)) {
            for (size_t b = 0; b < p->hx.size(); ++b)
                if (!p->tbox[b])
                    HCHECK(launch_interp_lines<R>(p->m, dxf + b, p->hx[b].n, p->at<int>(L.counters) + 1, p->til.T,
                                                  p->at<unsigned char>(L.rec), L.rec_bytes,
                                                  p->at<int>(L.cell_start), p->at<R>(L.outs), s));
        } else if (p->any_lines) {
            Tiling t = p->til;
            t.ring = use_ring(p, t);
            HCHECK(launch_interp<R>(p->m, false, dxf, p->at<SItem>(L.items), p->nitems,
                                    p->at<int>(L.counters) + 1, t, p->at<unsigned char>(L.rec), L.rec_bytes,
                                    p->at<int>(L.cell_start), p->at<R>(L.outs), s));
        }
    }
    {
        PhaseTimer t(p, HPNFFT_PH_SCATTER);
        HCHECK(launch_scatter<R>(p->at<R>(L.outs), p->at<int>(L.ipos), p->Mtot, f, s));
    }
    return HPNFFT_OK;
}

template <typename R>
int run_backward(hpnfft_plan_s *p, const void *f, const void *gfhat, void *grad_f, void *grad_x)
{
    const Layout &L = p->L;
    hipStream_t s = p->stream;
    const Xform *dxf = p->at<Xform>(L.xf);
    {
        PhaseTimer t(p, HPNFFT_PH_ZERO);
        HCHECK(launch_zero(p->ws + L.outs, L.outs_bytes, s));
    }
    int rc = run_to_grid<R>(p, gfhat);
    if (rc) return rc;
    {
        PhaseTimer t(p, HPNFFT_PH_GRAD);
        if (p->det())
            HCHECK(launch_interp_det<R>(p->m, true, dxf, p->B, p->Mtot, p->at<unsigned char>(L.rec), L.rec_bytes,
                                        p->at<R>(L.outs), p->cus, s));
        else if (p->any_box)
            HCHECK(launch_interp_box<R>(p->m, true, dxf, p->at<SItem>(L.bitems), p->nbitems,
                                        p->at<int>(L.counters) + 1, p->max_cells, p->at<unsigned char>(L.rec),
                                        L.rec_bytes, p->at<int>(L.cell_start), p->at<R>(L.outs), s));
        if (p->any_lines)
            HCHECK(launch_interp<R>(p->m, true, dxf, p->at<SItem>(L.items), p->nitems,
                                    p->at<int>(L.counters) + 1, p->til, p->at<unsigned char>(L.rec), L.rec_bytes,
                                    p->at<int>(L.cell_start), p->at<R>(L.outs), s));
    }
    {
        PhaseTimer t(p, HPNFFT_PH_GRAD_FIN);
        HCHECK(launch_grad_finish<R>(p->at<R>(L.outs), f, p->at<int>(L.ipos), p->Mtot, p->hx[0].flat, grad_f,
                                     grad_x, s));
    }
    return HPNFFT_OK;
}

// Smallest even grid edge >= v whose FFT factors are in {2, 3, 5, 7}.
int smooth_even_at_least(int v)
{
    int e = std::max(2, v + (v & 1));
    while (!is_smooth(e)) e += 2;
    return e;
}

// d < 3 (single transforms): the 3 - d leading dims are flat, with N_t = 1,
// every point at 0 and a unit-impulse window, so the three-dimensional
// kernels compute the d-dimensional transform exactly (their grid edge there
// is the smallest even smooth size >= 2m that the sweeps accept).
int create_common(hpnfft_plan_s **out, int B, const int64_t *N, const int64_t *M, double sigma, int m,
                  int window, int precision, unsigned flags, int dims = 3)
{
    if (!out || B < 1 || !N || !M) return HPNFFT_EINVAL;
    *out = nullptr;
    if (window < HPNFFT_KAISER_BESSEL || window > HPNFFT_SINC_POWER) return HPNFFT_EINVAL;
    if (precision != HPNFFT_F64 && precision != HPNFFT_F32) return HPNFFT_EINVAL;
    if (m < 1 || m > kMaxWindowM) return HPNFFT_EINVAL;
    if (flags & ~(HPNFFT_WITH_GRADIENT | HPNFFT_DETERMINISTIC)) return HPNFFT_EINVAL;
    if (!(sigma >= 1.0) || !std::isfinite(sigma)) return HPNFFT_EINVAL;
    hpnfft_plan_s *p = new (std::nothrow) hpnfft_plan_s();
    if (!p) return HPNFFT_ENOMEM;
    p->B = B;
    p->m = m;
    p->prec = precision;
    p->window = window;
    p->sigma = sigma;
    p->flags = flags;
    p->wp = window_params(window, m, sigma);
    p->hx.resize(B);
    p->keys.resize(B);
    long long Mtot = 0, Ftot = 0;
    const int flat = 3 - dims;
    for (int b = 0; b < B; ++b) {
        Xform &X = p->hx[b];
        std::memset(&X, 0, sizeof(X));
        X.flat = flat;
        if (M[b] < 1) { delete p; return HPNFFT_EINVAL; }
        for (int t = 0; t < flat; ++t) {
            X.N[t] = 1;
            X.n[t] = smooth_even_at_least(2 * m);
            p->maxn = std::max(p->maxn, X.n[t]);
        }
        for (int d = flat; d < 3; ++d) {
            int64_t Nt = N[dims * b + (d - flat)];
            if (Nt < 2 || Nt % 2 != 0 || Nt > kMaxN) { delete p; return HPNFFT_EINVAL; }
            double nv = sigma * (double)Nt;
            long nt = std::lround(nv);
            if (std::fabs(nv - (double)nt) > 1e-9 * nv || nt % 2 != 0 || !is_smooth(nt) || nt < 2 * m ||
                nt > kMaxN || nt < Nt) {
                delete p;
                return HPNFFT_EINVAL;
            }
            X.N[d] = (int)Nt;
            X.n[d] = (int)nt;
            p->maxn = std::max(p->maxn, (int)nt);
        }
        X.M = M[b];
        X.poff = Mtot;
        X.foff = Ftot;
        Mtot += M[b];
        Ftot += (long long)X.N[0] * X.N[1] * X.N[2];
    }
    if (Mtot >= (1LL << 31)) { delete p; return HPNFFT_EINVAL; }
    p->Mtot = Mtot;
    p->Ftot = Ftot;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
            p->cus = cus;
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
            // "gfx950:sramecc+:xnack-" -> "gfx950"
            size_t k = 0;
            while (k + 1 < sizeof(p->arch) && prop.gcnArchName[k] && prop.gcnArchName[k] != ':') {
                p->arch[k] = prop.gcnArchName[k];
                ++k;
            }
            p->arch[k] = 0;
        }
    }
    choose_methods(p);
    p->til = default_tiling(p);
    build_layout(p);
    prepare_host_tables(p);
    hlog("plan: B=%d m=%d %s sigma=%g first n=%dx%dx%d M=%lld tiles T=%d Zs=%d threads=%d workspace %zu B", B, m,
         precision == HPNFFT_F32 ? "f32" : "f64", sigma, p->hx[0].n[0], p->hx[0].n[1], p->hx[0].n[2],
         (long long)p->Mtot, p->til.T, p->til.Zs, p->til.threads, p->L.total);
    *out = p;
    return HPNFFT_OK;
}

}  // namespace

// ===========================================================================
extern "C" {

const char *hpnfft_strerror(int status)
{
    switch (status) {
    case HPNFFT_OK: return "success";
    case HPNFFT_EINVAL: return "invalid argument";
    case HPNFFT_EDOMAIN: return "point outside [-1/2,1/2)^d or not finite";
    case HPNFFT_ENOMEM: return "out of memory or workspace too small";
    case HPNFFT_EHIP: return "HIP runtime error";
    case HPNFFT_ESTATE: return "call out of order";
    case HPNFFT_ESIZE: return "input exceeds the library's fixed scratch capacity";
    default: return "unknown status";
    }
}

int hpnfft_plan_create(hpnfft_plan *out, int d, const int64_t *N, int64_t M, double sigma, int m, int window,
                       int precision, unsigned flags)
{
    if (d < 1 || d > 3) return HPNFFT_EINVAL;
    return create_common(out, 1, N, &M, sigma, m, window, precision, flags, d);
}

int hpnfft_batch_create(hpnfft_batch *out, int B, const int64_t *N, const int64_t *M, double sigma, int m,
                        int window, int precision, unsigned flags)
{
    return create_common(out, B, N, M, sigma, m, window, precision, flags);
}

int hpnfft_plan_destroy(hpnfft_plan p)
{
    if (!p) return HPNFFT_OK;
    // (teardown: a failure leaves nothing to undo)
    if (!p->recs.empty()) (void)hipStreamSynchronize(p->stream);
    drop_records(p);
    for (hipEvent_t e : p->pool) (void)hipEventDestroy(e);
    drop_graph(p);
    if (p->res_ev) {
        (void)hipEventSynchronize(p->res_ev);
        (void)hipEventDestroy(p->res_ev);
    }
    if (p->hres) (void)hipHostFree(p->hres);
    delete p;
    return HPNFFT_OK;
}

int hpnfft_set_stream(hpnfft_plan p, void *stream)
{
    if (!p) return HPNFFT_EINVAL;
    p->stream = (hipStream_t)stream;
    return HPNFFT_OK;
}

int hpnfft_set_tiles(hpnfft_plan p, int tile, int slab, int threads)
{
    if (!p) return HPNFFT_EINVAL;
    Tiling t = p->til;
    if (tile) t.T = tile;
    if (slab) t.Zs = slab;
    if (threads) t.threads = threads;
    if (!tiling_fits(p, t)) return HPNFFT_EINVAL;
    drop_graph(p);
    p->til = t;
    build_layout(p);
    p->have_ws = false;
    p->have_points = false;
    return HPNFFT_OK;
}

int hpnfft_set_method(hpnfft_plan p, int method)
{
    if (!p || method < HPNFFT_METHOD_AUTO || method > HPNFFT_METHOD_BOXES) return HPNFFT_EINVAL;
    if (p->det() && method == HPNFFT_METHOD_LINES) return HPNFFT_EINVAL;  // deterministic plans use boxes
    drop_graph(p);
    p->method = method;
    choose_methods(p);
    p->til = default_tiling(p);
    build_layout(p);
    p->have_ws = false;
    p->have_points = false;
    return HPNFFT_OK;
}

int hpnfft_get_method(hpnfft_plan p, int *method)
{
    if (!p || !method) return HPNFFT_EINVAL;
    *method = p->boxes ? HPNFFT_METHOD_BOXES : (p->any_box ? HPNFFT_METHOD_MIXED : HPNFFT_METHOD_LINES);
    return HPNFFT_OK;
}

int hpnfft_get_tiles(hpnfft_plan p, int *tile, int *slab, int *threads)
{
    if (!p) return HPNFFT_EINVAL;
    if (tile) *tile = p->til.T;
    if (slab) *slab = p->til.Zs;
    if (threads) *threads = p->til.threads;
    return HPNFFT_OK;
}

int hpnfft_workspace_size(hpnfft_plan p, size_t *bytes)
{
    if (!p || !bytes) return HPNFFT_EINVAL;
    *bytes = p->L.total;
    return HPNFFT_OK;
}

int hpnfft_set_workspace(hpnfft_plan p, void *dev_ptr, size_t bytes)
{
    if (!p || !dev_ptr) return HPNFFT_EINVAL;
    if (((uintptr_t)dev_ptr) % 256) return HPNFFT_EINVAL;
    if (bytes < p->L.total) return HPNFFT_ENOMEM;
    drop_graph(p);
    p->ws = (char *)dev_ptr;
    p->ws_bytes = bytes;
    p->have_points = false;
    int rc = upload_tables(p);
    p->have_ws = rc == HPNFFT_OK;
    return rc;
}

static int set_points_any(hpnfft_plan p, const double *x, const float *x32)
{
    if (!p || (!x && !x32)) return HPNFFT_EINVAL;
    if (!p->have_ws) return HPNFFT_ESTATE;
    drop_graph(p);
    p->have_points = false;
    int rc;
    {
        PhaseTimer t(p, HPNFFT_PH_SET_POINTS);
        rc = bin_points(p, x, x32);
    }
    p->have_points = rc == HPNFFT_OK;
    hlog("set_points: status %d, %d work items, staging hint %d points", rc, p->nitems, p->til.cap_hint);
    return rc;
}

int hpnfft_set_points(hpnfft_plan p, const double *x) { return set_points_any(p, x, nullptr); }
int hpnfft_set_points_f32(hpnfft_plan p, const float *x) { return set_points_any(p, nullptr, x); }
int hpnfft_batch_set_points(hpnfft_batch p, const double *x) { return set_points_any(p, x, nullptr); }

int hpnfft_adjoint(hpnfft_plan p, const void *f, void *fhat)
{
    if (!p || !f || !fhat) return HPNFFT_EINVAL;
    if (!p->have_points) return HPNFFT_ESTATE;
    return p->prec == HPNFFT_F32 ? run_adjoint<float>(p, f, fhat) : run_adjoint<double>(p, f, fhat);
}

int hpnfft_forward(hpnfft_plan p, const void *fhat, void *f)
{
    if (!p || !f || !fhat) return HPNFFT_EINVAL;
    if (!p->have_points) return HPNFFT_ESTATE;
    return p->prec == HPNFFT_F32 ? run_forward<float>(p, fhat, f) : run_forward<double>(p, fhat, f);
}

int hpnfft_batch_adjoint(hpnfft_batch p, const void *f, void *fhat) { return hpnfft_adjoint(p, f, fhat); }
int hpnfft_batch_forward(hpnfft_batch p, const void *fhat, void *f) { return hpnfft_forward(p, fhat, f); }

int hpnfft_adjoint_backward(hpnfft_plan p, const void *f, const void *gfhat, void *grad_f, void *grad_x)
{
    if (!p || !gfhat) return HPNFFT_EINVAL;
    if (!p->grad()) return HPNFFT_EINVAL;
    if (grad_x && !f) return HPNFFT_EINVAL;
    if (!p->have_points) return HPNFFT_ESTATE;
    if (!grad_f && !grad_x) return HPNFFT_OK;
    return p->prec == HPNFFT_F32 ? run_backward<float>(p, f, gfhat, grad_f, grad_x)
                                 : run_backward<double>(p, f, gfhat, grad_f, grad_x);
}

int hpnfft_ewald_recip(hpnfft_plan p, const void *S, double L, double alpha, double *energy_dev, void *gbar)
{
    if (!p || !S || !energy_dev || p->B != 1) return HPNFFT_EINVAL;
    if (!(L > 0.0) || !(alpha > 0.0)) return HPNFFT_EINVAL;
    if (!p->have_ws) return HPNFFT_ESTATE;
    const Xform &X = p->hx[0];
    double *part = p->at<double>(p->L.ewald);
    int nb = (int)(((long long)X.N[0] * X.N[1] * X.N[2] + 255) / 256);
    hipError_t e = p->prec == HPNFFT_F32
                       ? launch_ewald<float>(S, X, L, alpha, part, nb, energy_dev, gbar, p->stream)
                       : launch_ewald<double>(S, X, L, alpha, part, nb, energy_dev, gbar, p->stream);
    return hip_status(e);
}

int hpnfft_ewald_real(const double *r, const double *q, int64_t M, double L, double alpha, double rcut,
                      double *energy_dev, double *forces_dev, double *scratch_dev, void *stream)
{
    if (!r || !q || !energy_dev || !scratch_dev || M < 1) return HPNFFT_EINVAL;
    if (!(L > 0.0) || !(alpha > 0.0) || !(rcut > 0.0) || rcut > 0.5 * L) return HPNFFT_EINVAL;
    return hip_status(launch_ewald_real(r, q, M, L, alpha, rcut, scratch_dev, energy_dev, forces_dev,
                                        (hipStream_t)stream));
}

}  // extern "C"

namespace {
// Cells per box edge for the cell-list sum: side L / nc >= rcut, at least 3
// (the 27 neighbours are then distinct cells), at most kMaxCellEdge.
constexpr int kMaxCellEdge = 512;
int cell_edge(double L, double rcut)
{
    if (!(L > 0.0) || !(rcut > 0.0) || !std::isfinite(L / rcut)) return 0;
    const double q = std::floor(L / rcut);
    if (q < 3.0) return 0;
    return q > kMaxCellEdge ? kMaxCellEdge : (int)q;
}
}  // namespace

extern "C" {

int hpnfft_ewald_real_cells_workspace(int64_t M, double L, double rcut, size_t *bytes)
{
    if (!bytes || M < 1 || M >= (1LL << 31)) return HPNFFT_EINVAL;
    const int nc = cell_edge(L, rcut);
    if (!nc) return HPNFFT_EINVAL;
    *bytes = cells_layout(M, nc).total;
    return HPNFFT_OK;
}

int hpnfft_ewald_real_cells(const double *r, const double *q, int64_t M, double L, double alpha, double rcut,
                            double *energy_dev, double *forces_dev, void *workspace, size_t bytes, void *stream)
{
    if (!r || !q || !energy_dev || !workspace || M < 1 || M >= (1LL << 31)) return HPNFFT_EINVAL;
    if (!(alpha > 0.0) || ((uintptr_t)workspace) % 256) return HPNFFT_EINVAL;
    const int nc = cell_edge(L, rcut);
    if (!nc) return HPNFFT_EINVAL;
    if (bytes < cells_layout(M, nc).total) return HPNFFT_ENOMEM;
    return hip_status(launch_ewald_cells(r, q, M, L, alpha, rcut, nc, static_cast<unsigned char *>(workspace),
                                         energy_dev, forces_dev, (hipStream_t)stream));
}

int hpnfft_ewald_real_static(const double *r, const double *q, int64_t M, double L, double alpha, double rcut,
                             double *energy_dev, double *forces_dev, void *stream)
{
    if (!r || !q || !energy_dev || M < 1) return HPNFFT_EINVAL;
    if (!(L > 0.0) || !(alpha > 0.0) || !(rcut > 0.0) || rcut > 0.5 * L) return HPNFFT_EINVAL;
    if (M > hpnfft_ewald_real_static_max_ions()) {
        hlog("ewald_real_static: %lld ions exceed the static scratch (at most %lld)", (long long)M,
             (long long)hpnfft_ewald_real_static_max_ions());
        return HPNFFT_ESIZE;
    }
    double *part = nullptr;
    const int rc = static_scratch(&part);
    if (rc != HPNFFT_OK) return rc;
    return hip_status(launch_ewald_real(r, q, M, L, alpha, rcut, part, energy_dev, forces_dev, (hipStream_t)stream));
}

int64_t hpnfft_ewald_real_static_max_ions(void) { return (int64_t)kStaticScratchDoubles * kEwaldRealTile; }

int hpnfft_check_points(const double *x, int64_t M, int d, int64_t *first_bad)
{
    if (first_bad) *first_bad = -1;
    if (M < 0 || d < 1 || d > 3 || (M > 0 && !x)) return HPNFFT_EINVAL;
    for (int64_t j = 0; j < M; ++j)
        for (int t = 0; t < d; ++t) {
            const double v = x[j * d + t];
            if (!(v >= -0.5 && v < 0.5)) {  // NaN fails both comparisons
                if (first_bad) *first_bad = j;
                return HPNFFT_EDOMAIN;
            }
        }
    return HPNFFT_OK;
}

int hpnfft_copy(void *dst, const void *src, size_t bytes, void *stream)
{
    if ((!dst || !src) && bytes) return HPNFFT_EINVAL;
    if (((uintptr_t)dst | (uintptr_t)src) % 16) return HPNFFT_EINVAL;
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    return hip_status(launch_copy(dst, src, bytes, cus, (hipStream_t)stream));
}

int hpnfft_plan_info(hpnfft_plan p, int64_t *n_out, int64_t *M_out)
{
    if (!p) return HPNFFT_EINVAL;
    if (n_out)
        for (int d = p->hx[0].flat; d < 3; ++d) n_out[d - p->hx[0].flat] = p->hx[0].n[d];
    if (M_out) *M_out = p->Mtot;
    return HPNFFT_OK;
}

int hpnfft_batch_offsets(hpnfft_batch p, int b, int64_t *point_offset, int64_t *freq_offset)
{
    if (!p || b < 0 || b >= p->B) return HPNFFT_EINVAL;
    if (point_offset) *point_offset = p->hx[b].poff;
    if (freq_offset) *freq_offset = p->hx[b].foff;
    return HPNFFT_OK;
}

int hpnfft_batch_capture(hpnfft_batch p, const void *f, void *fhat)
{
    if (!p || !f || !fhat) return HPNFFT_EINVAL;
    if (!p->have_points) return HPNFFT_ESTATE;
    if (!p->stream) return HPNFFT_EINVAL;  // capture needs a non-default stream
    drop_graph(p);
    // attribute setup outside the capture: one eager run; no timing events
    // inside the graph
    const unsigned prof = p->prof;
    p->prof = 0;
    int rc = hpnfft_adjoint(p, f, fhat);
    if (rc) {
        p->prof = prof;
        return rc;
    }
    HCHECK(hipStreamSynchronize(p->stream));
    HCHECK(hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal));
    rc = hpnfft_adjoint(p, f, fhat);
    p->prof = prof;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(p->stream, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return HPNFFT_EHIP;
    p->graph = g;
    HCHECK(hipGraphInstantiate(&p->gexec, g, nullptr, nullptr, 0));
    return HPNFFT_OK;
}

int hpnfft_batch_launch(hpnfft_batch p)
{
    if (!p) return HPNFFT_EINVAL;
    if (!p->gexec) return HPNFFT_ESTATE;
    return hip_status(hipGraphLaunch(p->gexec, p->stream));
}

int hpnfft_autotune(hpnfft_plan p, void *scratch_f, void *scratch_fhat, int *tile, int *slab, int *threads)
{
    if (!p || !scratch_f || !scratch_fhat) return HPNFFT_EINVAL;
    if (!p->have_points) return HPNFFT_ESTATE;
    drop_graph(p);
    // candidates that fit the attached workspace
    // (line method: tile edge, slab depth, threads; box method: box edges)
    std::vector<Tiling> cand;
    std::vector<Tiling> grid;
    if (p->boxes) {
        for (int T : {8, 12, 16, 20, 24, 32})
            for (int Zs : {8, 12, 16, 20, 24, 32}) grid.push_back(Tiling{T, Zs, 512});
    } else {
        for (int T : {4, 6, 8, 12, 16})
            for (int Zs : {8, 16, 24, 32})
                for (int th : {512, 1024}) grid.push_back(Tiling{T, Zs, th});
    }
    for (const Tiling &t : grid) {
        if (!tiling_fits(p, t)) continue;
        Tiling keep = p->til;
        p->til = t;
        build_layout(p);
        size_t need = p->L.total;
        p->til = keep;
        build_layout(p);
        if (need <= p->ws_bytes) cand.push_back(t);
    }
    // The stored float64 points sit at the same workspace offset in every
    // layout (build_layout), so a candidate re-bins them where they are.
    auto install = [&](Tiling t) -> int {
        p->til = t;
        build_layout(p);
        int rc = upload_tables(p);
        if (rc) return rc;
        rc = bin_points(p, nullptr, nullptr);
        p->have_points = rc == HPNFFT_OK;
        return rc;
    };
    const std::string key = tune_key(p);
    Tiling cached{};
    if (tune_cache_get(key, &cached)) {
        bool ok = false;
        for (const Tiling &t : cand) ok |= t.T == cached.T && t.Zs == cached.Zs && t.threads == cached.threads;
        if (ok) {
            hlog("autotune: cache hit %s -> T=%d Zs=%d threads=%d", key.c_str(), cached.T, cached.Zs,
                 cached.threads);
            int rc = install(cached);
            if (tile) *tile = cached.T;
            if (slab) *slab = cached.Zs;
            if (threads) *threads = cached.threads;
            return rc;
        }
    }
    Tiling best = p->til;
    double best_t = 1e30;
    hipEvent_t e0, e1;
    HCHECK(hipEventCreate(&e0));
    HCHECK(hipEventCreate(&e1));
    // one round: the adjoint, then the forward, or for gradient plans the
    // backward that their users run instead.  Their point outputs go to the
    // workspace's sorted-values array (the next adjoint's gather rewrites
    // it), never back into scratch_f: fed back, the values would grow round
    // by round to inf and NaN.
    auto round = [&]() {
        void *outp = p->ws + p->L.fs;
        return hpnfft_adjoint(p, scratch_f, scratch_fhat) == 0 &&
               (p->grad() ? hpnfft_adjoint_backward(p, scratch_f, scratch_fhat, outp, nullptr) == 0
                          : hpnfft_forward(p, scratch_fhat, outp) == 0);
    };
    for (const Tiling &t : cand) {
        if (install(t)) continue;
        bool ok = true;
        for (int w = 0; w < 2 && ok; ++w) ok = round();
        if (!ok) continue;
        ok = hipEventRecord(e0, p->stream) == hipSuccess;
        for (int r = 0; r < 3 && ok; ++r) ok = round();
        float ms = 0;
        ok = ok && hipEventRecord(e1, p->stream) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
             hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
        hlog("autotune: T=%d Zs=%d threads=%d %.4f ms per round", t.T, t.Zs, t.threads, ok ? ms / 3 : -1.0);
        if (ok && ms < best_t) {
            best_t = ms;
            best = t;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    int rc = install(best);
    if (rc == HPNFFT_OK) tune_cache_put(key, best);
    if (tile) *tile = best.T;
    if (slab) *slab = best.Zs;
    if (threads) *threads = best.threads;
    return rc;
}

int hpnfft_profile(hpnfft_plan p, int enable)
{
    return hpnfft_profile_phases(p, enable ? (1u << HPNFFT_NPHASES) - 1u : 0u);
}

int hpnfft_profile_phases(hpnfft_plan p, unsigned mask)
{
    if (!p) return HPNFFT_EINVAL;
    if (!p->recs.empty()) HCHECK(hipStreamSynchronize(p->stream));
    drop_records(p);
    p->prof = mask & ((1u << HPNFFT_NPHASES) - 1u);
    return HPNFFT_OK;
}

int hpnfft_profile_read(hpnfft_plan p, double *ms, int64_t *counts)
{
    if (!p) return HPNFFT_EINVAL;
    if (!p->recs.empty()) HCHECK(hipEventSynchronize(p->recs.back().b));
    for (auto &r : p->recs) {
        float t = 0.f;
        HCHECK(hipEventElapsedTime(&t, r.a, r.b));
        if (ms) ms[r.phase] += t;
        if (counts) counts[r.phase] += 1;
    }
    drop_records(p);
    return HPNFFT_OK;
}

const char *hpnfft_phase_name(int phase)
{
    static const char *names[HPNFFT_NPHASES] = {"set_points", "zero",   "gather", "spread", "fft_a0",
                                                "fft_a1",     "fft_a2", "fft_f0", "fft_f1", "fft_f2",
                                                "interp",     "scatter", "grad_interp", "grad_finish"};
    return (phase >= 0 && phase < HPNFFT_NPHASES) ? names[phase] : "";
}

int hpnfft_window_eval(int window, int m, double sigma, int64_t count, const double *t, double *phi, double *dphi)
{
    if (window < HPNFFT_KAISER_BESSEL || window > HPNFFT_SINC_POWER) return HPNFFT_EINVAL;
    if (m < 1 || m > kMaxWindowM || !(sigma >= 1.0) || count < 0 || (count && (!t || !phi))) return HPNFFT_EINVAL;
    const WindowParams w = window_params(window, m, sigma);
    for (int64_t i = 0; i < count; ++i) {
        double v, d;
        win_eval(w, t[i], &v, &d);
        phi[i] = v;
        if (dphi) dphi[i] = d;
    }
    return HPNFFT_OK;
}

int hpnfft_window_error_bound(int window, int m, double sigma, double *bound)
{
    if (window < HPNFFT_KAISER_BESSEL || window > HPNFFT_SINC_POWER) return HPNFFT_EINVAL;
    if (m < 1 || m > kMaxWindowM || !(sigma > 1.0) || !bound) return HPNFFT_EINVAL;
    *bound = window_error_bound(window, m, sigma);
    return HPNFFT_OK;
}

int hpnfft_window_rolloff(int window, int m, double sigma, int64_t n, int64_t N, double *out)
{
    if (window < HPNFFT_KAISER_BESSEL || window > HPNFFT_SINC_POWER) return HPNFFT_EINVAL;
    if (m < 1 || m > kMaxWindowM || !(sigma >= 1.0) || n < 2 || N < 1 || N > n || !out) return HPNFFT_EINVAL;
    const WindowParams w = window_params(window, m, sigma);
    for (int64_t i = 0; i < N; ++i) out[i] = 1.0 / window_phihat(w, (long)(i - N / 2), (long)n);
    return HPNFFT_OK;
}

}  // extern "C"
