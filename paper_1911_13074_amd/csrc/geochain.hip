// geochain.hip -- host side of the C ABI declared in include/geochain.h:
// argument validation, dtype/op dispatch, per-(device, stream) workspaces
// and the launch drivers for fixed chains (Eq. 4) and reconstruction
// (Eq. 5).  Every step of the chain runs in the kernels of chain_block.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "geochain.h"
#include "chain_block.hpp"

namespace geochain {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

static int fail(int status, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return status;
}

#define GC_HIP(call)                                                              \
    do {                                                                          \
        hipError_t e_ = (call);                                                   \
        if (e_ != hipSuccess)                                                     \
            return fail(GC_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

static size_t elem_size(gc_dtype d) {
    switch (d) {
        case GC_U8: return 1;
        case GC_F32: return 4;
        case GC_F64: return 8;
    }
    return 0;
}

// Byte extent [lo, hi) touched by an image of this shape.
static std::pair<uintptr_t, uintptr_t> extent(const void *p, const gc_shape &s, size_t es) {
    uintptr_t lo = (uintptr_t)p;
    if (s.width == 0 || s.height == 0) return {lo, lo};
    uintptr_t hi = lo + ((uint64_t)(s.height - 1) * (uint64_t)s.pitch + (uint64_t)s.width) * es;
    return {lo, hi};
}

static bool overlap(std::pair<uintptr_t, uintptr_t> a, std::pair<uintptr_t, uintptr_t> b) {
    return a.first < b.second && b.first < a.second;
}

static int validate_shape(gc_dtype dtype, const gc_shape &s) {
    if (elem_size(dtype) == 0) return fail(GC_ERR_INVALID_ARG, "unknown dtype %d", (int)dtype);
    if (s.width < 0 || s.height < 0) return fail(GC_ERR_INVALID_ARG, "negative image size");
    if (s.pitch < s.width) return fail(GC_ERR_INVALID_ARG, "pitch %lld < width %lld",
                                       (long long)s.pitch, (long long)s.width);
    if (s.width > (1 << 30) || s.height > (1 << 30))
        return fail(GC_ERR_UNSUPPORTED, "image sides above 2^30 are not supported");
    return GC_OK;
}

// marker/mask/out checks shared by the geodesic entry points.
static int validate_images(gc_dtype dtype, const void *marker, const void *mask, const void *out,
                           const gc_shape &s) {
    int st = validate_shape(dtype, s);
    if (st != GC_OK) return st;
    const bool empty = s.width == 0 || s.height == 0;
    if (!empty && (!marker || !out)) return fail(GC_ERR_INVALID_ARG, "null image pointer");
    const size_t es = elem_size(dtype);
    if (!empty && mask) {
        if (overlap(extent(out, s, es), extent(mask, s, es)))
            return fail(GC_ERR_ALIAS, "out overlaps mask");
    }
    if (!empty && out != marker && overlap(extent(out, s, es), extent(marker, s, es)))
        return fail(GC_ERR_ALIAS, "out partially overlaps marker");
    return GC_OK;
}

// ---------------------------------------------------------------------------
// tuning
// ---------------------------------------------------------------------------
static std::mutex g_tune_mu;
static int g_tune_k = 0;      // 0 = built-in
static int g_tune_tile = -1;  // -1 = built-in

enum { FAM_128 = 0, FAM_64 = 1, NUM_FAMS = 2 };

template <typename T, int FAM> struct Family;
// 128 x 128 region: 2 columns per lane; 8 waves of 16 rows (16 waves of 8
// rows for f64, whose registers are twice as wide).
template <typename T> struct Family<T, FAM_128> {
    static constexpr int CW = 2;
    static constexpr int RPW = sizeof(T) == 8 ? 8 : 16;
    static constexpr int NW = sizeof(T) == 8 ? 16 : 8;
};
// 64 x 64 region for small images: 1 column per lane, 8 waves of 8 rows.
template <typename T> struct Family<T, FAM_64> {
    static constexpr int CW = 1;
    static constexpr int RPW = 8;
    static constexpr int NW = 8;
};

static int region_side(int fam) { return fam == FAM_128 ? 128 : 64; }

struct Plan1 {
    int fam;
    int k;
};

// Built-in choice of tile family and steps per launch.
static Plan1 choose_plan(const gc_shape &s, int64_t n, bool detect) {
    Plan1 p;
    const int64_t side = std::max(s.width, s.height);
    p.fam = side >= 384 ? FAM_128 : FAM_64;
    p.k = p.fam == FAM_128 ? 32 : 16;
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        if (g_tune_tile >= 0 && g_tune_tile < NUM_FAMS) p.fam = g_tune_tile;
        if (g_tune_k > 0) p.k = g_tune_k;
    }
    const int kmax = (region_side(p.fam) - 16) / 2;  // keep a core of >= 16
    p.k = std::max(1, std::min(p.k, kmax));
    if (detect) p.k = std::min(p.k, 32);
    if (n > 0 && n < p.k) p.k = (int)n;
    return p;
}

// ---------------------------------------------------------------------------
// workspaces, one per (device, stream)
// ---------------------------------------------------------------------------
struct Workspace {
    void *buf = nullptr;
    size_t bytes = 0;
    uint32_t *words = nullptr;      // device change words
    uint32_t *host_words = nullptr; // pinned mirror
    size_t nwords = 0;
};

static std::mutex g_ws_mu;
static std::map<std::pair<int, void *>, Workspace> g_ws;

static int get_workspace(void *stream, size_t bytes, size_t nwords, Workspace **out) {
    int dev = 0;
    GC_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> g(g_ws_mu);
    Workspace &w = g_ws[{dev, stream}];
    if (w.bytes < bytes) {
        if (w.buf) {
            GC_HIP(hipStreamSynchronize((hipStream_t)stream));
            GC_HIP(hipFree(w.buf));
            w.buf = nullptr;
            w.bytes = 0;
        }
        if (hipMalloc(&w.buf, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return fail(GC_ERR_NO_MEMORY, "workspace of %zu bytes", bytes);
        }
        w.bytes = bytes;
    }
    if (w.nwords < nwords) {
        if (w.words) {
            GC_HIP(hipStreamSynchronize((hipStream_t)stream));
            GC_HIP(hipFree(w.words));
            GC_HIP(hipHostFree(w.host_words));
            w.words = nullptr;
            w.host_words = nullptr;
            w.nwords = 0;
        }
        if (hipMalloc((void **)&w.words, nwords * 4) != hipSuccess) {
            (void)hipGetLastError();
            return fail(GC_ERR_NO_MEMORY, "change words");
        }
        if (hipHostMalloc((void **)&w.host_words, nwords * 4, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return fail(GC_ERR_NO_MEMORY, "pinned change words");
        }
        w.nwords = nwords;
    }
    *out = &w;
    return GC_OK;
}

__global__ void fill_words_kernel(uint32_t *p, int n, uint32_t v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// measurement hook: HIP events around every launch while enabled
// ---------------------------------------------------------------------------
struct ProfRec {
    hipEvent_t start, stop;
    int steps;
};
static std::mutex g_prof_mu;
static bool g_prof_on = false;
static std::vector<ProfRec> g_prof_recs;
static std::vector<hipEvent_t> g_prof_pool;

static hipEvent_t prof_event() {
    if (!g_prof_pool.empty()) {
        hipEvent_t e = g_prof_pool.back();
        g_prof_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

static void prof_clear() {
    for (auto &r : g_prof_recs) {
        if (r.start) g_prof_pool.push_back(r.start);
        if (r.stop) g_prof_pool.push_back(r.stop);
    }
    g_prof_recs.clear();
}

// Bracket one launch; returns the index of its record or -1.
static int prof_begin(hipStream_t st, int steps) {
    std::lock_guard<std::mutex> g(g_prof_mu);
    if (!g_prof_on) return -1;
    ProfRec r{prof_event(), prof_event(), steps};
    if (!r.start || !r.stop) return -1;
    (void)hipEventRecord(r.start, st);
    g_prof_recs.push_back(r);
    return (int)g_prof_recs.size() - 1;
}

static void prof_end(int idx, hipStream_t st) {
    if (idx < 0) return;
    std::lock_guard<std::mutex> g(g_prof_mu);
    if (idx < (int)g_prof_recs.size()) (void)hipEventRecord(g_prof_recs[idx].stop, st);
}

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------
using LaunchFn = void (*)(const BlockArgs &, int grid, hipStream_t);

template <typename T, int OP, int MODE, bool DETECT, int FAM>
static void launch_block(const BlockArgs &a, int grid, hipStream_t st) {
    using F = Family<T, FAM>;
    hipLaunchKernelGGL((chain_block_kernel<T, OP, MODE, DETECT, F::CW, F::RPW, F::NW>),
                       dim3(grid), dim3(64 * F::NW), 0, st, a);
}

template <typename T, int OP, int MODE, bool DETECT>
static LaunchFn pick_fam(int fam) {
    return fam == FAM_128 ? &launch_block<T, OP, MODE, DETECT, FAM_128>
                          : &launch_block<T, OP, MODE, DETECT, FAM_64>;
}

template <typename T>
static LaunchFn pick_t(int op, int mode, bool detect, int fam) {
    if (op == OP_DILATE) {
        if (mode == MODE_GEODESIC)
            return detect ? pick_fam<T, OP_DILATE, MODE_GEODESIC, true>(fam)
                          : pick_fam<T, OP_DILATE, MODE_GEODESIC, false>(fam);
        return pick_fam<T, OP_DILATE, MODE_PLAIN, false>(fam);
    }
    if (mode == MODE_GEODESIC)
        return detect ? pick_fam<T, OP_ERODE, MODE_GEODESIC, true>(fam)
                      : pick_fam<T, OP_ERODE, MODE_GEODESIC, false>(fam);
    return pick_fam<T, OP_ERODE, MODE_PLAIN, false>(fam);
}

static LaunchFn pick_launch(gc_dtype d, int op, int mode, bool detect, int fam) {
    switch (d) {
        case GC_U8: return pick_t<uint8_t>(op, mode, detect, fam);
        case GC_F32: return pick_t<float>(op, mode, detect, fam);
        case GC_F64: return pick_t<double>(op, mode, detect, fam);
    }
    return nullptr;
}

struct Geometry {
    int core_x, core_y, tiles_x, tiles;
};

static Geometry geometry(const gc_shape &s, int fam, int k) {
    Geometry g;
    const int side = region_side(fam);
    g.core_x = side - 2 * k;
    g.core_y = side - 2 * k;
    g.tiles_x = (int)((s.width + g.core_x - 1) / g.core_x);
    const int tiles_y = (int)((s.height + g.core_y - 1) / g.core_y);
    g.tiles = g.tiles_x * tiles_y;
    return g;
}

static int copy_image(void *dst, const void *src, const gc_shape &s, size_t es, hipStream_t st) {
    if (dst == src || s.width == 0 || s.height == 0) return GC_OK;
    GC_HIP(hipMemcpy2DAsync(dst, s.pitch * es, src, s.pitch * es, s.width * es, s.height,
                            hipMemcpyDeviceToDevice, st));
    return GC_OK;
}

// ---------------------------------------------------------------------------
// fixed-length chains
// ---------------------------------------------------------------------------
static int run_chain(gc_dtype dtype, int op, int mode, const void *src, const void *mask, void *out,
                     const gc_shape &s, int64_t n, void *stream) {
    if (n < 0) return fail(GC_ERR_INVALID_ARG, "n_steps < 0");
    const bool empty = s.width == 0 || s.height == 0;
    const size_t es = elem_size(dtype);
    hipStream_t st = (hipStream_t)stream;
    if (empty) return GC_OK;
    if (n == 0) return copy_image(out, src, s, es, st);

    const Plan1 p = choose_plan(s, n, false);
    // launches: L-1 of p.k steps and a last one with the remainder
    std::vector<int> ks;
    for (int64_t left = n; left > 0; left -= p.k) ks.push_back((int)std::min<int64_t>(p.k, left));
    // In place with an odd number of launches would make the first launch
    // write the buffer it reads: split the first launch (or copy first).
    bool copy_first = false;
    if (src == out && (ks.size() % 2 == 1)) {
        if (ks[0] >= 2) {
            const int a = ks[0] / 2;
            ks.insert(ks.begin(), a);
            ks[1] -= a;
        } else {
            copy_first = true;
        }
    }
    Workspace *ws = nullptr;
    const size_t bytes = (size_t)((s.height - 1) * s.pitch + s.width) * es;
    int rc = get_workspace(stream, bytes, 0, &ws);
    if (rc != GC_OK) return rc;

    const void *cur = src;
    if (copy_first) {
        rc = copy_image(ws->buf, src, s, es, st);
        if (rc != GC_OK) return rc;
        cur = ws->buf;
        // now reading from ws: the single launch writes out
    }
    const size_t L = ks.size();
    for (size_t i = 0; i < L; ++i) {
        void *dst = ((L - 1 - i) % 2 == 0) ? out : ws->buf;
        if (copy_first) dst = out;  // L == 1 here
        const Geometry g = geometry(s, p.fam, ks[i]);
        BlockArgs a{};
        a.src = cur;
        a.mask = mask;
        a.dst = dst;
        a.width = (int32_t)s.width;
        a.height = (int32_t)s.height;
        a.pitch = s.pitch;
        a.k = ks[i];
        a.core_x = g.core_x;
        a.core_y = g.core_y;
        a.tiles_x = g.tiles_x;
        LaunchFn fn = pick_launch(dtype, op, mode, false, p.fam);
        const int pr = prof_begin(st, ks[i]);
        fn(a, g.tiles, st);
        prof_end(pr, st);
        GC_HIP(hipGetLastError());
        cur = dst;
    }
    return GC_OK;
}

// ---------------------------------------------------------------------------
// reconstruction
// ---------------------------------------------------------------------------
static int run_reconstruct(gc_dtype dtype, int op, const void *marker, const void *mask, void *out,
                           const gc_shape &s, int64_t max_steps, int64_t *steps_out, void *stream) {
    const size_t es = elem_size(dtype);
    hipStream_t st = (hipStream_t)stream;
    if (steps_out) *steps_out = 0;
    if (s.width == 0 || s.height == 0) return GC_OK;
    const Plan1 p = choose_plan(s, max_steps > 0 ? max_steps : 0, true);
    const int k = p.k;
    constexpr int MAX_GROUP = 64;
    Workspace *ws = nullptr;
    const size_t bytes = (size_t)((s.height - 1) * s.pitch + s.width) * es;
    int rc = get_workspace(stream, bytes, MAX_GROUP + 1, &ws);
    if (rc != GC_OK) return rc;
    LaunchFn fn = pick_launch(dtype, op, MODE_GEODESIC, true, p.fam);

    int64_t total = 0;       // steps executed that changed something
    int64_t blocks = 0;      // launches issued so far (sets the ping-pong parity)
    const void *cur = marker;
    const void *result = marker;
    int group = 4;
    bool converged = false;

    auto make_args = [&](const void *src, void *dst, int kk, uint32_t *word, const uint32_t *prev,
                         uint32_t prev_full) {
        const Geometry g = geometry(s, p.fam, kk);
        BlockArgs a{};
        a.src = src;
        a.mask = mask;
        a.dst = dst;
        a.width = (int32_t)s.width;
        a.height = (int32_t)s.height;
        a.pitch = s.pitch;
        a.k = kk;
        a.core_x = g.core_x;
        a.core_y = g.core_y;
        a.tiles_x = g.tiles_x;
        a.change_word = word;
        a.prev_word = prev;
        a.prev_full = prev_full;
        return std::make_pair(a, g.tiles);
    };

    while (!converged) {
        const int64_t budget = max_steps < 0 ? INT64_MAX : max_steps - total;
        if (budget <= 0) break;
        // plan this group's launches
        std::vector<int> ks;
        int64_t planned = 0;
        for (int j = 0; j < group && planned < budget; ++j) {
            const int kk = (int)std::min<int64_t>(k, budget - planned);
            ks.push_back(kk);
            planned += kk;
        }
        const int G = (int)ks.size();
        hipLaunchKernelGGL(fill_words_kernel, dim3(1), dim3(128), 0, st, ws->words, G, 0u);
        GC_HIP(hipGetLastError());
        std::vector<const void *> dsts(G);
        for (int j = 0; j < G; ++j) {
            void *dst = (blocks % 2 == 0) ? ws->buf : out;
            const uint32_t *prev = j > 0 ? ws->words + (j - 1) : nullptr;
            const uint32_t prev_full = j > 0 ? (uint32_t)((1ull << ks[j - 1]) - 1) : 0u;
            auto ag = make_args(cur, dst, ks[j], ws->words + j, prev, prev_full);
            const int pr = prof_begin(st, ks[j]);
            fn(ag.first, ag.second, st);
            prof_end(pr, st);
            GC_HIP(hipGetLastError());
            dsts[j] = dst;
            cur = dst;
            ++blocks;
        }
        GC_HIP(hipMemcpyAsync(ws->host_words, ws->words, G * 4, hipMemcpyDeviceToHost, st));
        GC_HIP(hipStreamSynchronize(st));
        for (int j = 0; j < G; ++j) {
            const uint32_t full = (uint32_t)((1ull << ks[j]) - 1);
            const uint32_t wrd = ws->host_words[j];
            result = dsts[j];
            if (wrd == full) {
                total += ks[j];
                continue;
            }
            total += __builtin_popcount(wrd);
            converged = true;
            break;
        }
        group = std::min(group * 2, MAX_GROUP);
    }

    if (!converged) {
        // The cap was hit with every step changing: one more look decides
        // whether the last state is already stable.
        void *dst = (result == (const void *)ws->buf) ? out : ws->buf;
        hipLaunchKernelGGL(fill_words_kernel, dim3(1), dim3(128), 0, st, ws->words, 1, 0u);
        GC_HIP(hipGetLastError());
        auto ag = make_args(result, dst, 1, ws->words, nullptr, 0u);
        fn(ag.first, ag.second, st);
        GC_HIP(hipGetLastError());
        GC_HIP(hipMemcpyAsync(ws->host_words, ws->words, 4, hipMemcpyDeviceToHost, st));
        GC_HIP(hipStreamSynchronize(st));
        converged = ws->host_words[0] == 0;
        // result still names the chain of max_steps steps (dst equals it if
        // converged, and is one step further otherwise).
    }
    if (result != out) {
        rc = copy_image(out, result, s, es, st);
        if (rc != GC_OK) return rc;
    }
    if (steps_out) *steps_out = total;
    if (!converged) return fail(GC_ERR_NOT_CONVERGED, "reconstruction did not converge in %lld steps",
                                (long long)max_steps);
    return GC_OK;
}

}  // namespace geochain

using namespace geochain;

extern "C" {

int gc_version(void) { return 100; }

const char *gc_status_string(int status) {
    switch (status) {
        case GC_OK: return "GC_OK";
        case GC_ERR_INVALID_ARG: return "GC_ERR_INVALID_ARG";
        case GC_ERR_UNSUPPORTED: return "GC_ERR_UNSUPPORTED";
        case GC_ERR_ALIAS: return "GC_ERR_ALIAS";
        case GC_ERR_NO_MEMORY: return "GC_ERR_NO_MEMORY";
        case GC_ERR_HIP: return "GC_ERR_HIP";
        case GC_ERR_NOT_CONVERGED: return "GC_ERR_NOT_CONVERGED";
    }
    return "GC_ERR_UNKNOWN";
}

const char *gc_last_error(void) { return g_last_error.c_str(); }

static int geodesic_chain(gc_dtype dtype, int op, const void *marker, const void *mask, void *out,
                          gc_shape shape, int64_t n_steps, void *stream) {
    g_last_error.clear();
    int rc = validate_images(dtype, marker, mask, out, shape);
    if (rc != GC_OK) return rc;
    if (!(shape.width == 0 || shape.height == 0) && !mask)
        return fail(GC_ERR_INVALID_ARG, "null mask");
    if (n_steps < 0) return fail(GC_ERR_INVALID_ARG, "n_steps < 0");
    return run_chain(dtype, op, MODE_GEODESIC, marker, mask, out, shape, n_steps, stream);
}

int gc_geodesic_dilate_chain(gc_dtype dtype, const void *marker, const void *mask, void *out,
                             gc_shape shape, int64_t n_steps, void *hip_stream) {
    return geodesic_chain(dtype, OP_DILATE, marker, mask, out, shape, n_steps, hip_stream);
}

int gc_geodesic_erode_chain(gc_dtype dtype, const void *marker, const void *mask, void *out,
                            gc_shape shape, int64_t n_steps, void *hip_stream) {
    return geodesic_chain(dtype, OP_ERODE, marker, mask, out, shape, n_steps, hip_stream);
}

static int plain_chain(gc_dtype dtype, int op, const void *in, void *out, gc_shape shape,
                       int64_t n_steps, void *stream) {
    g_last_error.clear();
    int rc = validate_images(dtype, in, nullptr, out, shape);
    if (rc != GC_OK) return rc;
    if (n_steps < 0) return fail(GC_ERR_INVALID_ARG, "n_steps < 0");
    return run_chain(dtype, op, MODE_PLAIN, in, nullptr, out, shape, n_steps, stream);
}

int gc_dilate_chain(gc_dtype dtype, const void *in, void *out, gc_shape shape, int64_t n_steps,
                    void *hip_stream) {
    return plain_chain(dtype, OP_DILATE, in, out, shape, n_steps, hip_stream);
}

int gc_erode_chain(gc_dtype dtype, const void *in, void *out, gc_shape shape, int64_t n_steps,
                   void *hip_stream) {
    return plain_chain(dtype, OP_ERODE, in, out, shape, n_steps, hip_stream);
}

static int reconstruct(gc_dtype dtype, int op, const void *marker, const void *mask, void *out,
                       gc_shape shape, int64_t max_steps, int64_t *steps_out, void *stream) {
    g_last_error.clear();
    int rc = validate_images(dtype, marker, mask, out, shape);
    if (rc != GC_OK) return rc;
    if (!(shape.width == 0 || shape.height == 0) && !mask)
        return fail(GC_ERR_INVALID_ARG, "null mask");
    return run_reconstruct(dtype, op, marker, mask, out, shape, max_steps, steps_out, stream);
}

int gc_reconstruct_by_dilation(gc_dtype dtype, const void *marker, const void *mask, void *out,
                               gc_shape shape, int64_t max_steps, int64_t *steps_out,
                               void *hip_stream) {
    return reconstruct(dtype, OP_DILATE, marker, mask, out, shape, max_steps, steps_out, hip_stream);
}

int gc_reconstruct_by_erosion(gc_dtype dtype, const void *marker, const void *mask, void *out,
                              gc_shape shape, int64_t max_steps, int64_t *steps_out,
                              void *hip_stream) {
    return reconstruct(dtype, OP_ERODE, marker, mask, out, shape, max_steps, steps_out, hip_stream);
}

int gc_profile_enable(int on) {
    std::lock_guard<std::mutex> g(g_prof_mu);
    g_prof_on = on != 0;
    if (!g_prof_on) prof_clear();
    return GC_OK;
}

int gc_profile_read(double *kernel_ms, int64_t *launches, int64_t *steps) {
    g_last_error.clear();
    std::lock_guard<std::mutex> g(g_prof_mu);
    double total = 0.0;
    int64_t n = 0, nsteps = 0;
    for (auto &r : g_prof_recs) {
        GC_HIP(hipEventSynchronize(r.stop));
        float ms = 0.f;
        GC_HIP(hipEventElapsedTime(&ms, r.start, r.stop));
        total += ms;
        ++n;
        nsteps += r.steps;
    }
    prof_clear();
    if (kernel_ms) *kernel_ms = total;
    if (launches) *launches = n;
    if (steps) *steps = nsteps;
    return GC_OK;
}

int gc_set_tuning(int32_t block_steps, int32_t tile) {
    if (block_steps < 0 || block_steps > 63) return fail(GC_ERR_INVALID_ARG, "block_steps out of range");
    if (tile < -1 || tile >= NUM_FAMS) return fail(GC_ERR_INVALID_ARG, "tile family out of range");
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune_k = block_steps;
    g_tune_tile = tile;
    return GC_OK;
}

}  // extern "C"
