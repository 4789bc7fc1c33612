// geochain.hip -- host side of the C ABI declared in include/geochain.h:
// argument validation, dtype/op dispatch, per-(device, stream) workspaces
// and the launch drivers for fixed chains (Eq. 4) and reconstruction
// (Eq. 5).  Every step of the chain runs in the kernels of chain_block.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "geochain.h"
#include "chain_block.hpp"
#include "chain_launch.hpp"
#include "persistent.hpp"
#include "grad_block.hpp"
#include "operators.hpp"
#include "qdt_block.hpp"
#include "window_hgw.hpp"

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

// Fault injection for tests of the error path: with the environment
// variable GEOCHAIN_INJECT_HIP_FAULT set to some text, every checked HIP
// call (GC_HIP below) whose source text contains it is not made and fails
// with GC_ERR_HIP instead.  Read once, at the first checked call.
static const char *inject_pattern() {
    static const char *p = [] {
        const char *e = getenv("GEOCHAIN_INJECT_HIP_FAULT");
        return (e && *e) ? e : (const char *)nullptr;
    }();
    return p;
}

static bool inject_fault(const char *call_text) {
    const char *p = inject_pattern();
    return p != nullptr && strstr(call_text, p) != nullptr;
}

#define GC_HIP(call)                                                              \
    do {                                                                          \
        if (inject_fault(#call))                                                  \
            return fail(GC_ERR_HIP, "%s failed: injected fault", #call);          \
        hipError_t e_ = (call);                                                   \
        if (e_ != hipSuccess)                                                     \
            return fail(GC_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// Finite test on the bit pattern (exponent not all ones), which no
// floating-point option of the compiler can fold away.
static bool finite_bits(double v) {
    uint64_t b;
    memcpy(&b, &v, sizeof b);
    return ((b >> 52) & 0x7FFu) != 0x7FFu;
}

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
    // Sides up to 2^25 keep every launch below 2^32 work-items (the line
    // kernels of the large-window path run one 64-lane workgroup per image
    // line); 2^36 pixels (a 64 GiB u8 image) keep tile counts in 32 bits.
    if (s.width > (int64_t(1) << 25) || s.height > (int64_t(1) << 25))
        return fail(GC_ERR_UNSUPPORTED, "image sides above 2^25 are not supported (%lld x %lld)",
                    (long long)s.width, (long long)s.height);
    if (s.width * s.height > (int64_t(1) << 36))
        return fail(GC_ERR_UNSUPPORTED, "images above 2^36 pixels are not supported (%lld x %lld)",
                    (long long)s.width, (long long)s.height);
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
// workspaces, one per (device, stream)
// ---------------------------------------------------------------------------
struct Workspace {
    void *buf = nullptr;
    size_t bytes = 0;
    uint32_t *words = nullptr;      // device change words
    uint32_t *host_words = nullptr; // pinned, mapped mirror (host address)
    uint32_t *host_words_dev = nullptr; // the same memory as the device sees it
    size_t nwords = 0;
    void *partials = nullptr;       // PARTIALS_MAX per-workgroup extrema (operators)
    void *buf2 = nullptr;           // images of composed operators (granulometry)
    size_t bytes2 = 0;
    // A HIP graph recorded by stream capture keeps the addresses of buf and
    // buf2 as they were during the capture.  Once a capture has used them
    // they are never freed: when a later call needs more room, the old
    // buffer is retired (kept allocated until the process ends) and a new
    // one takes its place, so replays never touch freed memory.
    bool captured = false;
    bool captured2 = false;
};

static std::mutex g_ws_mu;
static std::map<std::pair<int, void *>, Workspace> g_ws;
static std::vector<void *> g_retired;   // buffers a recorded graph may still use

// Whether work enqueued on the stream now is being recorded into a graph.
static int stream_capturing(void *stream, bool *capturing) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    GC_HIP(hipStreamIsCapturing((hipStream_t)stream, &cs));
    *capturing = cs != hipStreamCaptureStatusNone;
    return GC_OK;
}

// Replaces a workspace buffer that must grow: freed after the stream's work
// is done, or retired if a capture has used it.
static int grow_release(void *stream, void **buf, size_t *bytes, bool *captured, bool capturing) {
    if (capturing)
        return fail(GC_ERR_UNSUPPORTED, "the stream's workspace would have to grow during stream capture "
                                        "(%zu bytes now); make an uncaptured call of this size first", *bytes);
    if (!*buf) return GC_OK;
    if (*captured) {
        g_retired.push_back(*buf);
    } else {
        GC_HIP(hipStreamSynchronize((hipStream_t)stream));
        GC_HIP(hipFree(*buf));
    }
    *buf = nullptr;
    *bytes = 0;
    *captured = false;
    return GC_OK;
}

static int get_workspace(void *stream, size_t bytes, size_t nwords, Workspace **out) {
    int dev = 0;
    GC_HIP(hipGetDevice(&dev));
    bool capturing = false;
    {
        const int rc = stream_capturing(stream, &capturing);
        if (rc != GC_OK) return rc;
    }
    std::lock_guard<std::mutex> g(g_ws_mu);
    Workspace &w = g_ws[{dev, stream}];
    if (w.bytes < bytes) {
        const int rc = grow_release(stream, &w.buf, &w.bytes, &w.captured, capturing);
        if (rc != GC_OK) return rc;
        if (hipMalloc(&w.buf, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return fail(GC_ERR_NO_MEMORY, "workspace of %zu bytes", bytes);
        }
        w.bytes = bytes;
    }
    if (capturing && bytes > 0) w.captured = true;
    if (w.nwords < nwords) {
        if (capturing) return fail(GC_ERR_UNSUPPORTED, "change words cannot be allocated during stream capture");
        if (w.words) {
            GC_HIP(hipStreamSynchronize((hipStream_t)stream));
            GC_HIP(hipFree(w.words));
            GC_HIP(hipHostFree(w.host_words));
            w.words = nullptr;
            w.host_words = nullptr;
            w.host_words_dev = nullptr;
            w.nwords = 0;
        }
        if (hipMalloc((void **)&w.words, nwords * 4) != hipSuccess) {
            (void)hipGetLastError();
            return fail(GC_ERR_NO_MEMORY, "change words");
        }
        if (hipHostMalloc((void **)&w.host_words, nwords * 4, hipHostMallocMapped | hipHostMallocCoherent) !=
            hipSuccess) {
            (void)hipGetLastError();
            return fail(GC_ERR_NO_MEMORY, "pinned change words");
        }
        GC_HIP(hipHostGetDevicePointer((void **)&w.host_words_dev, w.host_words, 0));
        w.nwords = nwords;
    }
    *out = &w;
    return GC_OK;
}

// Per-(device, stream) buffer of PARTIALS_MAX doubles for the extremum pass.
static int get_partials(void *stream, void **out) {
    int dev = 0;
    GC_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> g(g_ws_mu);
    Workspace &w = g_ws[{dev, stream}];
    if (!w.partials) {
        if (hipMalloc(&w.partials, PARTIALS_MAX * sizeof(double)) != hipSuccess) {
            (void)hipGetLastError();
            w.partials = nullptr;
            return fail(GC_ERR_NO_MEMORY, "extremum partials");
        }
    }
    *out = w.partials;
    return GC_OK;
}

// Per-(device, stream) second buffer for operators composed of several
// chains (run_chain keeps the first one for its ping-pong).
static int get_buf2(void *stream, size_t bytes, void **out) {
    int dev = 0;
    GC_HIP(hipGetDevice(&dev));
    bool capturing = false;
    {
        const int rc = stream_capturing(stream, &capturing);
        if (rc != GC_OK) return rc;
    }
    std::lock_guard<std::mutex> g(g_ws_mu);
    Workspace &w = g_ws[{dev, stream}];
    if (w.bytes2 < bytes) {
        const int rc = grow_release(stream, &w.buf2, &w.bytes2, &w.captured2, capturing);
        if (rc != GC_OK) return rc;
        if (hipMalloc(&w.buf2, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return fail(GC_ERR_NO_MEMORY, "operator workspace of %zu bytes", bytes);
        }
        w.bytes2 = bytes;
    }
    if (capturing && bytes > 0) w.captured2 = true;
    *out = w.buf2;
    return GC_OK;
}

__global__ void fill_words_kernel(uint32_t *p, int n, uint32_t v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Copies n device words into the mapped host mirror with system-scope
// stores: after the stream has been synchronised the host reads them
// directly, with no copy command.
__global__ void publish_words_kernel(const uint32_t *src, uint32_t *host_dst, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x)
        __hip_atomic_store(host_dst + i, src[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// The first n change words, read on the host (synchronises the stream).
static int read_words(Workspace *ws, int n, hipStream_t st) {
    hipLaunchKernelGGL(publish_words_kernel, dim3(1), dim3(64), 0, st, ws->words, ws->host_words_dev, n);
    GC_HIP(hipGetLastError());
    GC_HIP(hipStreamSynchronize(st));
    return GC_OK;
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

static int copy_image(void *dst, const void *src, const gc_shape &s, size_t es, hipStream_t st) {
    if (dst == src || s.width == 0 || s.height == 0) return GC_OK;
    GC_HIP(hipMemcpy2DAsync(dst, s.pitch * es, src, s.pitch * es, s.width * es, s.height,
                            hipMemcpyDeviceToDevice, st));
    return GC_OK;
}

// ---------------------------------------------------------------------------
// large windows: plain chains as one (2n+1)^2 window (van Herk / Gil-Werman)
// ---------------------------------------------------------------------------
static int g_window_min_steps = 0;   // 0: built-in threshold, -1: never
// Measured crossovers at 1024 x 1024 against the register-blocked chain:
// the window path takes 18-19 us (u8), 24-25 us (f32), 34-36 us (f64) at
// any n up to 183; the chain 19 / 20 / 25 us at 24 steps and 22 / 22 / 30 us
// at 32.  Below these many steps the chain is at least as fast.
static int window_min_steps_default(gc_dtype dtype) {
    switch (dtype) {
        case GC_U8: return 26;
        case GC_F32: return 34;
        default: return 38;
    }
}
constexpr size_t HGW_LDS_MAX = 65536;

// Padded positions per lane: odd (distinct LDS banks across lanes) and
// enough for the line plus n neutral pixels on each side; rounded up to a
// length the register kernel is compiled for when one fits.
static const int HGW_REG_SEGS[] = {9, 17, 25, 33, 49, 65};
static int64_t hgw_seg(int64_t length, int64_t n) {
    const int64_t s = ((length + 2 * n + 63) / 64) | 1;
    for (int r : HGW_REG_SEGS)
        if (s <= r) return r;
    return s;
}

// LDS of one line: g and h (register width) and the line itself.
static size_t hgw_lds_bytes(gc_dtype dtype, int64_t length, int64_t n) {
    const size_t rs = dtype == GC_F64 ? 8 : 4;
    return (size_t)hgw_seg(length, n) * 64 * 2 * rs + (size_t)length * elem_size(dtype);
}

static bool window_path(gc_dtype dtype, const gc_shape &s, int64_t n) {
    int thr;
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        thr = g_window_min_steps;
    }
    if (thr < 0) return false;
    if (thr == 0) thr = window_min_steps_default(dtype);
    if (n < thr) return false;
    const int64_t nr = std::min<int64_t>(n, s.width - 1), nc = std::min<int64_t>(n, s.height - 1);
    return hgw_lds_bytes(dtype, s.width, nr) <= HGW_LDS_MAX && hgw_lds_bytes(dtype, s.height, nc) <= HGW_LDS_MAX;
}

// One line per wave: the register kernel when a lane's segment fits it.
template <typename T, int OP>
static void hgw_rows(const HgwArgs &a, unsigned lines, size_t lds, hipStream_t st) {
    switch (a.seg) {
#define GC_HGW_REG(S_) \
    case S_: hipLaunchKernelGGL((hgw_rows_reg_kernel<T, OP, S_>), dim3(lines), dim3(64), lds, st, a); return;
        GC_HGW_REG(9)
        GC_HGW_REG(17)
        GC_HGW_REG(25)
        GC_HGW_REG(33)
        GC_HGW_REG(49)
        GC_HGW_REG(65)
#undef GC_HGW_REG
        default: hipLaunchKernelGGL((hgw_rows_kernel<T, OP>), dim3(lines), dim3(64), lds, st, a);
    }
}

// dst (height x width) = transpose of src (width x height).
template <typename T>
static void transpose(const T *src, T *dst, int64_t width, int64_t height, int64_t src_pitch, int64_t dst_pitch,
                      hipStream_t st) {
    const dim3 grid((unsigned)((width + 63) / 64), (unsigned)((height + 63) / 64));
    const bool vec = (uintptr_t)src % 16 == 0 && (uintptr_t)dst % 16 == 0 && (src_pitch * (int64_t)sizeof(T)) % 16 == 0 &&
                     (dst_pitch * (int64_t)sizeof(T)) % 16 == 0;
    if (vec)
        hipLaunchKernelGGL((transpose_kernel<T, true>), grid, dim3(256), 0, st, src, dst, (int32_t)width, (int32_t)height,
                           src_pitch, dst_pitch);
    else
        hipLaunchKernelGGL((transpose_kernel<T, false>), grid, dim3(256), 0, st, src, dst, (int32_t)width,
                           (int32_t)height, src_pitch, dst_pitch);
}

template <typename T, int OP>
static int run_window_t(const T *in, T *out, const gc_shape &s, int64_t n, void *stream) {
    using R = typename RegOf<T>::type;
    hipStream_t st = (hipStream_t)stream;
    const int64_t X = s.width, Y = s.height;
    // A window wider than the image clips to the whole line: radius X-1
    // (Y-1) gives the same result as any larger one.
    const int32_t nr = (int32_t)std::min<int64_t>(n, X - 1), nc = (int32_t)std::min<int64_t>(n, Y - 1);
    // temporaries with pitches rounded to 16 bytes (vector transposes)
    const int64_t per16 = 16 / (int64_t)sizeof(T);
    const int64_t px_ = (X + per16 - 1) / per16 * per16, py_ = (Y + per16 - 1) / per16 * per16;
    const size_t plane = ((size_t)(std::max(px_ * Y, py_ * X)) * sizeof(T) + 255) & ~(size_t)255;
    Workspace *ws = nullptr;
    int rc = get_workspace(stream, 2 * plane, 0, &ws);
    if (rc != GC_OK) return rc;
    T *ta = static_cast<T *>(ws->buf);
    T *tb = reinterpret_cast<T *>(static_cast<char *>(ws->buf) + plane);

    HgwArgs r{};
    r.src = in;
    r.dst = ta;
    r.length = (int32_t)X;
    r.lines = (int32_t)Y;
    r.src_pitch = s.pitch;
    r.dst_pitch = px_;
    r.n = nr;
    r.seg = (int32_t)hgw_seg(X, nr);
    int pr = prof_begin(st, 0);
    hgw_rows<T, OP>(r, (unsigned)Y, r.seg * 64 * 2 * sizeof(R) + X * sizeof(T), st);
    prof_end(pr, st);
    transpose(ta, tb, X, Y, px_, py_, st);
    HgwArgs c = r;
    c.src = tb;
    c.dst = ta;
    c.length = (int32_t)Y;
    c.lines = (int32_t)X;
    c.src_pitch = py_;
    c.dst_pitch = py_;
    c.n = nc;
    c.seg = (int32_t)hgw_seg(Y, nc);
    pr = prof_begin(st, 0);
    hgw_rows<T, OP>(c, (unsigned)X, c.seg * 64 * 2 * sizeof(R) + Y * sizeof(T), st);
    prof_end(pr, st);
    transpose(ta, out, Y, X, py_, s.pitch, st);
    GC_HIP(hipGetLastError());
    return GC_OK;
}

static int run_window(gc_dtype dtype, int op, const void *in, void *out, const gc_shape &s, int64_t n,
                      void *stream) {
    switch (dtype) {
        case GC_U8:
            return op == OP_DILATE ? run_window_t<uint8_t, OP_DILATE>((const uint8_t *)in, (uint8_t *)out, s, n, stream)
                                   : run_window_t<uint8_t, OP_ERODE>((const uint8_t *)in, (uint8_t *)out, s, n, stream);
        case GC_F32:
            return op == OP_DILATE ? run_window_t<float, OP_DILATE>((const float *)in, (float *)out, s, n, stream)
                                   : run_window_t<float, OP_ERODE>((const float *)in, (float *)out, s, n, stream);
        case GC_F64:
            return op == OP_DILATE ? run_window_t<double, OP_DILATE>((const double *)in, (double *)out, s, n, stream)
                                   : run_window_t<double, OP_ERODE>((const double *)in, (double *)out, s, n, stream);
    }
    return fail(GC_ERR_INVALID_ARG, "unknown dtype");
}

// ---------------------------------------------------------------------------
// fixed-length chains
// ---------------------------------------------------------------------------
// fixed_ws: a caller-chosen work buffer of fixed_bytes bytes in place of
// the stream's workspace (the entry point that allocates nothing); such
// calls also skip the measurement hook, whose events are allocated.
// Batches (n_images > 1): images of one shape at image_stride elements from
// each other, all advanced by the same launches (one workgroup per tile of
// every image).
static int copy_batch(void *dst, const void *src, const gc_shape &s, size_t es, hipStream_t st, int32_t n_images,
                      int64_t image_stride) {
    for (int32_t i = 0; i < n_images; ++i) {
        const size_t off = (size_t)i * (size_t)image_stride * es;
        const int rc = copy_image((char *)dst + off, (const char *)src + off, s, es, st);
        if (rc != GC_OK) return rc;
    }
    return GC_OK;
}

// MODE_MIXED (u8 and f32): erode_steps[i] != 0 makes step i an erosion,
// else a dilation; op is unused.
static int run_chain(gc_dtype dtype, int op, int mode, const void *src, const void *mask, void *out,
                     const gc_shape &s, int64_t n, void *stream, void *fixed_ws = nullptr,
                     size_t fixed_bytes = 0, int32_t n_images = 1, int64_t image_stride = 0,
                     const uint8_t *erode_steps = nullptr) {
    if (n < 0) return fail(GC_ERR_INVALID_ARG, "n_steps < 0");
    const bool mixed = mode == MODE_MIXED;
    if (mixed && (dtype == GC_F64 || erode_steps == nullptr))
        return fail(GC_ERR_UNSUPPORTED, "mixed chains take u8 or f32 images and a list of steps");
    const bool empty = s.width == 0 || s.height == 0 || n_images == 0;
    const size_t es = elem_size(dtype);
    hipStream_t st = (hipStream_t)stream;
    if (empty) return GC_OK;
    if (n_images == 1) image_stride = 0;
    if (n == 0) return copy_batch(out, src, s, es, st, n_images, image_stride);
    if (n_images == 1 && mode == MODE_PLAIN && window_path(dtype, s, n))
        return run_window(dtype, op, src, out, s, n, stream);

    const Plan1 p = mixed ? Plan1{FAM_128W, (int)std::min<int64_t>(32, n)} : choose_plan(s, n, false);
    // Launches: L0 - 1 of p.k steps and a last one with the remainder.  In
    // place with an odd number of launches would make the first launch
    // write the buffer it reads: split the first launch in two (or, if it
    // is a single step, copy first).  Computed per launch, with no list.
    const int64_t L0 = (n + p.k - 1) / p.k;
    const int k0 = (int)std::min<int64_t>(p.k, n);
    bool split = false, copy_first = false;
    if (src == out && L0 % 2 == 1) {
        if (k0 >= 2) split = true;
        else copy_first = true;
    }
    const int64_t L = L0 + (split ? 1 : 0);
    auto k_of = [&](int64_t i) -> int {
        if (split) {
            if (i == 0) return k0 / 2;
            if (i == 1) return k0 - k0 / 2;
            i -= 1;
        }
        return (int)std::min<int64_t>(p.k, n - i * p.k);
    };
    const size_t bytes = (size_t)((int64_t)(n_images - 1) * image_stride + (s.height - 1) * s.pitch + s.width) * es;
    {
        // tile counts of a launch stay in 32 bits
        const Geometry g = geometry(s, p.fam, p.k);   // the most tiles of any launch
        if ((int64_t)g.tiles * n_images > (int64_t)INT32_MAX)
            return fail(GC_ERR_UNSUPPORTED, "%d images of %d tiles each exceed 2^31 - 1 tiles", n_images, g.tiles);
    }
    void *work = fixed_ws;
    if (fixed_ws) {
        if (bytes > fixed_bytes)
            return fail(GC_ERR_UNSUPPORTED, "image needs %zu bytes of work buffer, the fixed one holds %zu", bytes,
                        fixed_bytes);
    } else {
        Workspace *ws = nullptr;
        const int rc = get_workspace(stream, bytes, 0, &ws);
        if (rc != GC_OK) return rc;
        work = ws->buf;
    }
    const bool hook = fixed_ws == nullptr;

    const void *cur = src;
    if (copy_first) {
        const int rc = copy_batch(work, src, s, es, st, n_images, image_stride);
        if (rc != GC_OK) return rc;
        cur = work;
    }
    int64_t step0 = 0;   // the launch's first step
    for (int64_t i = 0; i < L; ++i) {
        const int ki = k_of(i);
        // the last launch writes out; after a copy into the work buffer the
        // first launch reads it, and the alternation never writes the
        // buffer a launch reads
        void *dst = ((L - 1 - i) % 2 == 0) ? out : work;
        const Geometry g = geometry(s, p.fam, ki);
        BlockArgs a{};
        a.src = cur;
        a.mask = mask;
        a.dst = dst;
        a.width = (int32_t)s.width;
        a.height = (int32_t)s.height;
        a.pitch = s.pitch;
        a.k = ki;
        a.halo = ki;
        a.core_x = g.core_x;
        a.core_y = g.core_y;
        a.tiles_x = g.tiles_x;
        a.tiles_per_image = n_images > 1 ? g.tiles : 0;
        a.image_stride = image_stride;
        if (mixed)
            for (int j = 0; j < ki; ++j)
                if (erode_steps[step0 + j]) a.erode_bits |= uint64_t(1) << j;
        LaunchFn fn = mixed ? pick_mixed(dtype) : pick_launch(dtype, op, mode, false, p.fam);
        const int pr = hook ? prof_begin(st, ki) : -1;
        fn(a, g.tiles * n_images, st);
        if (hook) prof_end(pr, st);
        GC_HIP(hipGetLastError());
        cur = dst;
        step0 += ki;
    }
    return GC_OK;
}

// ---------------------------------------------------------------------------
// the chain entry point that allocates nothing
// ---------------------------------------------------------------------------
// Its ping-pong buffer: one array per device, held until the process ends.
// In host code the name `scratch` stands for the symbol, not for device
// memory; the device address comes from hipGetSymbolAddress, taken once per
// device with that device current, and only that address is ever passed on.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)16 << 20;
__device__ __align__(256) uint8_t scratch[NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[NOALLOC_MAX_DEVICES];

static int scratch_address(void **out) {
    int dev = 0;
    GC_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
        return fail(GC_ERR_UNSUPPORTED, "device ordinal %d beyond %d", dev, NOALLOC_MAX_DEVICES - 1);
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        GC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(GC_ERR_HIP, "hipGetSymbolAddress returned a null address");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
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
    // Launches per host check: start with 8 blocks (a few hundred steps, the
    // typical reconstruction length), then double; launches past the
    // convergence point exit at once.
    int group = 8;
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
        a.halo = kk;
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
        {
            const int wrc = read_words(ws, G, st);
            if (wrc != GC_OK) return wrc;
        }
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
        {
            const int wrc = read_words(ws, 1, st);
            if (wrc != GC_OK) return wrc;
        }
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

// ---------------------------------------------------------------------------
// reconstruction-based operators (Eq. 6-12)
// ---------------------------------------------------------------------------
enum { GOP_HMAX = 0, GOP_DOME = 1, GOP_HFILL = 2, GOP_RAOBJ = 3, GOP_OPEN_REC = 4 };

// 16-byte chunks need every row start of every image aligned to 16 bytes.
static bool rows_aligned16(const gc_shape &s, size_t es, const void *a, const void *b) {
    return (s.pitch * (int64_t)es) % 16 == 0 && (uintptr_t)a % 16 == 0 && (uintptr_t)b % 16 == 0;
}

template <typename T>
static PixelArgs<T> pixel_args(const gc_shape &s, const T *a, const T *b, T *out, bool vec) {
    PixelArgs<T> p{};
    p.a = a;
    p.b = b;
    p.out = out;
    p.width = (int32_t)s.width;
    p.height = (int32_t)s.height;
    p.pitch = s.pitch;
    const int64_t V = vec ? 16 / (int64_t)sizeof(T) : 1;
    p.chunks_per_row = (s.width + V - 1) / V;
    p.n_chunks = p.chunks_per_row * s.height;
    return p;
}

static int px_grid(int64_t n_chunks, int64_t cap) {
    return (int)std::max<int64_t>(1, std::min<int64_t>((n_chunks + PX_THREADS - 1) / PX_THREADS, cap));
}

template <typename T, int KIND, int OP>
static void px_launch(const PixelArgs<T> &p, bool vec, hipStream_t st) {
    const int grid = px_grid(p.n_chunks, 4096);
    if (vec)
        hipLaunchKernelGGL((pixel_kernel<T, KIND, OP, true>), dim3(grid), dim3(PX_THREADS), 0, st, p);
    else
        hipLaunchKernelGGL((pixel_kernel<T, KIND, OP, false>), dim3(grid), dim3(PX_THREADS), 0, st, p);
}

// Writes one extremum per workgroup to p.out; returns how many.
template <typename T, int OP>
static int extremum_launch(const PixelArgs<T> &p, bool vec, hipStream_t st) {
    const int grid = px_grid(p.n_chunks, PARTIALS_MAX);
    if (vec)
        hipLaunchKernelGGL((extremum_kernel<T, OP, true>), dim3(grid), dim3(PX_THREADS), 0, st, p);
    else
        hipLaunchKernelGGL((extremum_kernel<T, OP, false>), dim3(grid), dim3(PX_THREADS), 0, st, p);
    return grid;
}

// Marker pass, one reconstruction with f as the mask, and for DOME / RAOBJ
// the final difference f - rec.  out holds the marker, then the result.
template <typename T>
static int run_operator_t(gc_dtype dtype, int which, const T *f, T *out, const gc_shape &s, T h,
                          int64_t size, int64_t max_steps, int64_t *steps_out, void *stream) {
    hipStream_t st = (hipStream_t)stream;
    const bool vec = rows_aligned16(s, sizeof(T), f, out);
    int rec_op = OP_DILATE;
    if (which == GOP_HMAX || which == GOP_DOME) {
        PixelArgs<T> p = pixel_args<T>(s, f, nullptr, out, vec);
        p.h = h;
        px_launch<T, PX_SUB_SCALAR, OP_DILATE>(p, vec, st);
        GC_HIP(hipGetLastError());
    } else if (which == GOP_HFILL || which == GOP_RAOBJ) {
        void *partials = nullptr;
        int rc = get_partials(stream, &partials);
        if (rc != GC_OK) return rc;
        const PixelArgs<T> pe = pixel_args<T>(s, f, nullptr, (T *)partials, vec);
        PixelArgs<T> pb = pixel_args<T>(s, f, nullptr, out, vec);
        pb.partials = (const T *)partials;
        if (which == GOP_HFILL) {
            pb.n_partials = extremum_launch<T, OP_DILATE>(pe, vec, st);
            px_launch<T, PX_BORDER, OP_DILATE>(pb, vec, st);
            rec_op = OP_ERODE;
        } else {
            pb.n_partials = extremum_launch<T, OP_ERODE>(pe, vec, st);
            px_launch<T, PX_BORDER, OP_ERODE>(pb, vec, st);
        }
        GC_HIP(hipGetLastError());
    } else {
        int rc = run_chain(dtype, OP_ERODE, MODE_PLAIN, f, nullptr, out, s, size, stream);
        if (rc != GC_OK) return rc;
    }
    const int rrc = run_reconstruct(dtype, rec_op, out, f, out, s, max_steps, steps_out, stream);
    if (rrc != GC_OK && rrc != GC_ERR_NOT_CONVERGED) return rrc;
    if (which == GOP_DOME || which == GOP_RAOBJ) {
        px_launch<T, PX_SUB_IMAGE, OP_DILATE>(pixel_args<T>(s, f, out, out, vec), vec, st);
        GC_HIP(hipGetLastError());
    }
    return rrc;
}

// ---------------------------------------------------------------------------
// granulometry and alternating sequential filters (Eq. 16-20)
// ---------------------------------------------------------------------------
// G[s] = sum of gamma_s(f), s = 0..s_max.  The erosions are kept incremental
// (eps_s = eps_1(eps_{s-1}), the s-fold composition of Eq. 16), the
// dilations of each opening start from eps_s.  Each opening leaves its
// workgroup partials in a slot of its own; one launch per SUMS_PER_LAUNCH
// openings adds the slots' partials (then the slots are reused).
template <typename T>
static int run_granulometry_t(gc_dtype dtype, const T *f, const gc_shape &s, int s_max, double *G,
                              void *stream) {
    hipStream_t st = (hipStream_t)stream;
    const size_t npx = (size_t)((s.height - 1) * s.pitch + s.width);
    const size_t ext = (npx * sizeof(T) + 255) & ~(size_t)255;
    const size_t n_sums = (size_t)s_max + 1;
    const size_t sums_bytes = (n_sums * sizeof(double) + 255) & ~(size_t)255;
    void *b2 = nullptr;
    int rc = get_buf2(stream, 3 * ext + sums_bytes + (size_t)SUMS_PER_LAUNCH * PARTIALS_MAX * sizeof(double), &b2);
    if (rc != GC_OK) return rc;
    char *base = static_cast<char *>(b2);
    T *opened = reinterpret_cast<T *>(base);
    T *eroded[2] = {reinterpret_cast<T *>(base + ext), reinterpret_cast<T *>(base + 2 * ext)};
    double *sums = reinterpret_cast<double *>(base + 3 * ext);
    double *partials = reinterpret_cast<double *>(base + 3 * ext + sums_bytes);
    PartialCounts counts{};
    const T *eps = f;
    for (int sz = 0; sz <= s_max; ++sz) {
        const T *img = f;
        if (sz > 0) {
            T *next = eroded[sz % 2];
            rc = run_chain(dtype, OP_ERODE, MODE_PLAIN, eps, nullptr, next, s, 1, stream);
            if (rc != GC_OK) return rc;
            eps = next;
            rc = run_chain(dtype, OP_DILATE, MODE_PLAIN, eps, nullptr, opened, s, sz, stream);
            if (rc != GC_OK) return rc;
            img = opened;
        }
        const bool vec = rows_aligned16(s, sizeof(T), img, img);
        const PixelArgs<T> p = pixel_args<T>(s, img, nullptr, nullptr, vec);
        const int grid = px_grid(p.n_chunks, PARTIALS_MAX);
        const int b = sz % SUMS_PER_LAUNCH;
        double *slot = partials + (size_t)b * PARTIALS_MAX;
        if (vec)
            hipLaunchKernelGGL((sum_kernel<T, true>), dim3(grid), dim3(PX_THREADS), 0, st, p, slot);
        else
            hipLaunchKernelGGL((sum_kernel<T, false>), dim3(grid), dim3(PX_THREADS), 0, st, p, slot);
        counts.n[b] = grid;
        if (b == SUMS_PER_LAUNCH - 1 || sz == s_max)
            hipLaunchKernelGGL(sum_partials_kernel, dim3(b + 1), dim3(PX_THREADS), 0, st, (const double *)partials,
                               (int64_t)PARTIALS_MAX, counts, sums + (sz - b));
        GC_HIP(hipGetLastError());
    }
    std::vector<double> host(s_max + 1);
    GC_HIP(hipMemcpyAsync(host.data(), sums, (s_max + 1) * sizeof(double), hipMemcpyDeviceToHost, st));
    GC_HIP(hipStreamSynchronize(st));
    std::copy(host.begin(), host.end(), G);
    return GC_OK;
}

// phi_s(gamma_s(...)) as one list of plain chains; consecutive chains of the
// same direction are one chain of the summed length (delta_a of delta_b is
// delta_{a+b} by Eq. 4), so the sequence runs as E1 D2 E3 D4 ... D2S ES.
// u8 and f32: consecutive chains shorter than 64 steps that do not take the
// window path run as one mixed chain (a dilation or an erosion per step),
// 32 steps per launch whatever the chains' lengths.
static int run_asf(gc_dtype dtype, const void *f, void *out, const gc_shape &s, int s_max, void *stream) {
    const size_t es = elem_size(dtype);
    if (s_max == 0) return copy_image(out, f, s, es, (hipStream_t)stream);
    std::vector<std::pair<int, int64_t>> seq;
    auto push = [&](int op, int64_t n) {
        if (!seq.empty() && seq.back().first == op)
            seq.back().second += n;
        else
            seq.push_back({op, n});
    };
    for (int sz = 1; sz <= s_max; ++sz) {
        push(OP_ERODE, sz);   // gamma_s: erosions, then dilations
        push(OP_DILATE, sz);
        push(OP_DILATE, sz);  // phi_s: dilations, then erosions
        push(OP_ERODE, sz);
    }
    const void *cur = f;
    std::vector<uint8_t> run;   // steps of the pending mixed chain (1 = erosion)
    auto flush = [&]() -> int {
        if (run.empty()) return GC_OK;
        const int rc = run_chain(dtype, OP_DILATE, MODE_MIXED, cur, nullptr, out, s, (int64_t)run.size(), stream,
                                 nullptr, 0, 1, 0, run.data());
        run.clear();
        cur = out;
        return rc;
    };
    for (const auto &c : seq) {
        if (dtype != GC_F64 && c.second < 64 && !window_path(dtype, s, c.second)) {
            run.insert(run.end(), (size_t)c.second, (uint8_t)(c.first == OP_ERODE));
            if (run.size() >= ((size_t)1 << 16)) {
                const int rc = flush();
                if (rc != GC_OK) return rc;
            }
            continue;
        }
        int rc = flush();
        if (rc != GC_OK) return rc;
        rc = run_chain(dtype, c.first, MODE_PLAIN, cur, nullptr, out, s, c.second, stream);
        if (rc != GC_OK) return rc;
        cur = out;
    }
    return flush();
}

// ---------------------------------------------------------------------------
// quasi-distance transform (Eq. 13-15)
// ---------------------------------------------------------------------------
template <typename T, int PHASE, int CW, int RPW, int NW>
static void launch_qdt(const QdtArgs &qa, int grid, hipStream_t st) {
    // split like launch_block: the cores of r and d a tile updates are its own
    for (int t0 = 0; t0 < grid; t0 += MAX_TILES_PER_LAUNCH) {
        QdtArgs q = qa;
        q.b.tile0 = t0;
        hipLaunchKernelGGL((qdt_block_kernel<T, PHASE, CW, RPW, NW>), dim3(std::min(grid - t0, MAX_TILES_PER_LAUNCH)),
                           dim3(64 * NW), 0, st, q);
    }
}

struct QdtLayout {
    int rx, ry, k;  // region columns, rows; steps per launch
    void (*launch)(const QdtArgs &, int, hipStream_t);
};

// 128 x 128 regions (two columns per lane), k = 32; f64 keeps one column
// per lane (64 x 128, k = 16) so its residuals fit in registers.
template <typename T, int PHASE>
static QdtLayout qdt_layout() {
    if constexpr (sizeof(T) == 8) return {64, 128, 16, launch_qdt<T, PHASE, 1, 8, 16>};
    else return {128, 128, 32, launch_qdt<T, PHASE, 2, 8, 16>};
}

// Runs one phase, k steps per launch, until a step changes nothing.  The
// state starts in src0 and alternates between buf0 and buf1; *result is the
// buffer holding the final state and *changed the number of steps that
// changed a pixel.
static int run_qdt_phase(const QdtLayout &L, const gc_shape &s, const void *src0, void *buf0, void *buf1,
                         void *res, int32_t *dist, Workspace *ws, hipStream_t st, int64_t *changed,
                         const void **result) {
    constexpr int MAX_GROUP = 64;
    const int k = L.k;
    const int core_x = L.rx - 2 * k, core_y = L.ry - 2 * k;
    const int tiles_x = (int)((s.width + core_x - 1) / core_x);
    const int tiles = tiles_x * (int)((s.height + core_y - 1) / core_y);
    // Both chains stop changing within max(X, Y) - 1 steps; the bound only
    // guards the loop.
    const int64_t bound = 2 * std::max(s.width, s.height) + 2 * (int64_t)k * MAX_GROUP;
    const uint32_t full = (uint32_t)((1ull << k) - 1);
    int64_t total = 0, launched = 0;
    const void *cur = src0;
    *result = src0;
    int group = 8;
    for (bool done = false; !done;) {
        if (launched * k > bound) return fail(GC_ERR_HIP, "quasi-distance chain did not settle");
        hipLaunchKernelGGL(fill_words_kernel, dim3(1), dim3(128), 0, st, ws->words, group, 0u);
        GC_HIP(hipGetLastError());
        std::vector<const void *> dsts(group);
        for (int j = 0; j < group; ++j) {
            void *dst = (launched % 2 == 0) ? buf0 : buf1;
            QdtArgs qa{};
            qa.b.src = cur;
            qa.b.dst = dst;
            qa.b.width = (int32_t)s.width;
            qa.b.height = (int32_t)s.height;
            qa.b.pitch = s.pitch;
            qa.b.k = k;
            qa.b.halo = k;
            qa.b.core_x = core_x;
            qa.b.core_y = core_y;
            qa.b.tiles_x = tiles_x;
            qa.b.change_word = ws->words + j;
            qa.b.prev_word = j > 0 ? ws->words + (j - 1) : nullptr;
            qa.b.prev_full = full;
            qa.res = res;
            qa.dist = dist;
            qa.step0 = (int32_t)(launched * k);
            const int pr = prof_begin(st, k);
            L.launch(qa, tiles, st);
            prof_end(pr, st);
            GC_HIP(hipGetLastError());
            dsts[j] = dst;
            cur = dst;
            ++launched;
        }
        {
            const int wrc = read_words(ws, group, st);
            if (wrc != GC_OK) return wrc;
        }
        for (int j = 0; j < group; ++j) {
            const uint32_t wrd = ws->host_words[j];
            *result = dsts[j];
            if (wrd == full) {
                total += k;
                continue;
            }
            total += __builtin_popcount(wrd);
            done = true;
            break;
        }
        group = std::min(group * 2, MAX_GROUP);
    }
    *changed = total;
    return GC_OK;
}

template <typename T>
static int run_qdt_t(const T *f, int32_t *dist, T *residual, const gc_shape &s, bool lipschitz,
                     int64_t *erosion_steps, int64_t *eta_steps, void *stream) {
    hipStream_t st = (hipStream_t)stream;
    const size_t npx = (size_t)((s.height - 1) * s.pitch + s.width);
    const size_t ext_t = (npx * sizeof(T) + 255) & ~(size_t)255;
    const size_t ext_i = (npx * 4 + 255) & ~(size_t)255;
    Workspace *ws = nullptr;
    int rc = get_workspace(stream, std::max(3 * ext_t, ext_i), 65, &ws);
    if (rc != GC_OK) return rc;
    char *base = static_cast<char *>(ws->buf);
    T *res = residual ? residual : reinterpret_cast<T *>(base + 2 * ext_t);

    const void *state = nullptr;
    int64_t n_erode = 0;
    rc = run_qdt_phase(qdt_layout<T, QDT_ERODE>(), s, f, base, base + ext_t, res, dist, ws, st, &n_erode,
                       &state);
    if (rc != GC_OK) return rc;
    if (erosion_steps) *erosion_steps = n_erode;
    int64_t n_eta = 0;
    if (lipschitz) {
        const void *out = nullptr;
        rc = run_qdt_phase(qdt_layout<uint32_t, QDT_ETA>(), s, dist, base, dist, nullptr, nullptr, ws, st,
                           &n_eta, &out);
        if (rc != GC_OK) return rc;
        if (out != (const void *)dist) {
            rc = copy_image(dist, out, s, 4, st);
            if (rc != GC_OK) return rc;
        }
    }
    if (eta_steps) *eta_steps = n_eta;
    return GC_OK;
}

// ---------------------------------------------------------------------------
// persistent batched chains (plans)
// ---------------------------------------------------------------------------
struct PersistentFns {
    const void *kernel;  // for the occupancy query
    void (*launch)(const PersistentArgs &, int grid, hipStream_t);
    int threads;
};

template <typename T, int OP, int MODE, int FAM, bool DETECT = false>
static void launch_persistent(const PersistentArgs &a, int grid, hipStream_t st) {
    using F = Family<T, FAM>;
    hipLaunchKernelGGL((persistent_chain_kernel<T, OP, MODE, F::CW, F::RPW, F::NW, F::G, DETECT>), dim3(grid),
                       dim3(64 * F::NW), 0, st, a);
}

template <typename T, int OP, int MODE, int FAM, bool DETECT = false>
static PersistentFns persistent_fns_t() {
    using F = Family<T, FAM>;
    PersistentFns f;
    f.kernel = (const void *)&persistent_chain_kernel<T, OP, MODE, F::CW, F::RPW, F::NW, F::G, DETECT>;
    f.launch = &launch_persistent<T, OP, MODE, FAM, DETECT>;
    f.threads = 64 * F::NW;
    return f;
}

template <typename T, int OP, int MODE>
static PersistentFns persistent_fns_m(int fam) {
    switch (fam) {
        case FAM_64: return persistent_fns_t<T, OP, MODE, FAM_64>();
        case FAM_128W: return persistent_fns_t<T, OP, MODE, FAM_128W>();
        case FAM_96: return persistent_fns_t<T, OP, MODE, FAM_96>();
        case FAM_96W: return persistent_fns_t<T, OP, MODE, FAM_96W>();
        default: return persistent_fns_t<T, OP, MODE, FAM_128>();
    }
}

// Plans with run-to-stability items: change bits on, geodesic, 128 x 128
// regions of 16 waves (the built-in family).
template <typename T>
static PersistentFns persistent_fns_detect(int op) {
    return op == OP_DILATE ? persistent_fns_t<T, OP_DILATE, MODE_GEODESIC, FAM_128W, true>()
                           : persistent_fns_t<T, OP_ERODE, MODE_GEODESIC, FAM_128W, true>();
}

template <typename T>
static PersistentFns persistent_fns_d(int op, int mode, int fam) {
    if (op == OP_DILATE)
        return mode == MODE_GEODESIC ? persistent_fns_m<T, OP_DILATE, MODE_GEODESIC>(fam)
                                     : persistent_fns_m<T, OP_DILATE, MODE_PLAIN>(fam);
    return mode == MODE_GEODESIC ? persistent_fns_m<T, OP_ERODE, MODE_GEODESIC>(fam)
                                 : persistent_fns_m<T, OP_ERODE, MODE_PLAIN>(fam);
}

static PersistentFns persistent_fns(gc_dtype d, int op, int mode, int fam, bool detect) {
    if (detect) {
        switch (d) {
            case GC_U8: return persistent_fns_detect<uint8_t>(op);
            case GC_F32: return persistent_fns_detect<float>(op);
            case GC_F64: return persistent_fns_detect<double>(op);
        }
        return PersistentFns{};
    }
    switch (d) {
        case GC_U8: return persistent_fns_d<uint8_t>(op, mode, fam);
        case GC_F32: return persistent_fns_d<float>(op, mode, fam);
        case GC_F64: return persistent_fns_d<double>(op, mode, fam);
    }
    return PersistentFns{};
}

// Largest steps per block the persistent kernel accepts: the halo must not
// reach past the neighbouring tiles (k <= core = side - 2k).
static int persistent_kmax(int fam) { return region_side(fam) / 3; }
// Run-to-stability items in plans: steps per block and blocks per replay.
// Every block after an image's first unchanged step is wasted work and every
// replay a host wait; on 16 images of 65 to 648 steps, replays of 2 blocks of
// 20 steps took 3.7 ms, of 3 blocks 3.7, 4 blocks 4.2, 8 blocks 4.5 and 16
// blocks 5.6 (16 steps x 2 blocks 3.9, 24 x 2 3.8, 28 x 2 4.0).
constexpr int STAB_K = 20;
constexpr int STAB_BLOCKS = 2;
// Bound of one dependency wait in the batch kernel: 2 s of the 100 MHz
// clock, far beyond any wait of a launch that makes progress.
constexpr uint64_t PLAN_WAIT_TICKS = 200000000ull;

// Built-in steps per block for batches: with many items in flight the
// per-item latency is hidden, so a shallower block (less halo) wins.
static int default_persistent_k(int fam) {
    const int side = region_side(fam);
    return side == 128 ? 20 : side == 96 ? 16 : 12;
}

// ---- autotuner table ----
struct TuneKey {
    int dtype, op, geodesic, cw, ch;
    bool operator<(const TuneKey &o) const {
        return std::tie(dtype, op, geodesic, cw, ch) < std::tie(o.dtype, o.op, o.geodesic, o.cw, o.ch);
    }
};
struct TuneVal {
    int best_fam = FAM_128;
    int k[NUM_FAMS] = {};
    double rate[NUM_FAMS] = {};  // pixel-steps per second
};
static std::mutex g_autotune_mu;
static std::map<TuneKey, TuneVal> g_autotune;

static int ceil_log2(int64_t v) {
    int c = 0;
    while ((int64_t(1) << c) < v) ++c;
    return c;
}

static TuneKey tune_key(gc_dtype d, int op, int geodesic, int64_t w, int64_t h) {
    return TuneKey{(int)d, op, geodesic ? 1 : 0, ceil_log2(std::max<int64_t>(w, 1)),
                   ceil_log2(std::max<int64_t>(h, 1))};
}

}  // namespace geochain

struct gc_plan {
    int device = 0;
    gc_dtype dtype = GC_U8;
    int op = 0, mode = 0, fam = 0, max_k = 0;
    int32_t n_items = 0, grid = 0;
    int64_t px_steps = 0;
    std::vector<gc_item> items;
    geochain::PlanImage *images_d = nullptr;
    geochain::PlanItem *items_d = nullptr;
    uint32_t *words_d = nullptr;  // [0] ticket, [1] error, [2..] tile counters
    int64_t n_words = 0;
    void *ws = nullptr;
    uint32_t *error_h = nullptr;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t last_stream = nullptr;
    bool launched = false;
    // run-to-stability items (n_steps < 0): rounds of STAB_BLOCKS blocks of
    // STAB_K steps, the host deciding between graph replays
    std::vector<geochain::PlanImage> imgs_init;  // the image table as recorded
    std::vector<int> img_item;                   // plan image -> gc_item index
    std::vector<int> stab_imgs;                  // plan images that run to stability
    uint32_t *change_h = nullptr;                // pinned copy of their change words
    std::vector<int64_t> steps;                  // per gc_item, of the last launch
};

namespace geochain {

static void plan_free(gc_plan *p) {
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
    if (p->images_d) (void)hipFree(p->images_d);
    if (p->items_d) (void)hipFree(p->items_d);
    if (p->words_d) (void)hipFree(p->words_d);
    if (p->ws) (void)hipFree(p->ws);
    if (p->error_h) (void)hipHostFree(p->error_h);
    if (p->change_h) (void)hipHostFree(p->change_h);
    delete p;
}

struct PlanChoice {
    int fam;
    std::vector<int> k;  // per item
    int wgs_per_cu = 0;  // 0: as many as fit
};

// Tile family for the whole plan and steps per block for each item: from
// the autotuner when every item's size class has an entry, else built-in.
static PlanChoice choose_plan_batch(gc_dtype d, int op, int mode, const std::vector<gc_item> &items) {
    PlanChoice c;
    c.fam = FAM_128W;   // measured best for the 64-image uneven batch (k = 20, two workgroups per CU)
    int forced_k = 0, forced_fam = -1;
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        forced_k = g_tune_k;
        forced_fam = g_tune_tile;
    }
    std::vector<TuneVal> vals;
    bool all_tuned = true;
    {
        std::lock_guard<std::mutex> g(g_autotune_mu);
        for (const auto &it : items) {
            auto f = g_autotune.find(tune_key(d, op, mode == MODE_GEODESIC, it.shape.width, it.shape.height));
            if (f == g_autotune.end()) {
                all_tuned = false;
                vals.push_back(TuneVal{});
            } else {
                vals.push_back(f->second);
            }
        }
    }
    if (all_tuned && !items.empty()) {
        double best_t = 1e300;
        for (int fam = 0; fam < NUM_FAMS; ++fam) {
            double t = 0;
            bool ok = true;
            for (size_t i = 0; i < items.size(); ++i) {
                if (vals[i].rate[fam] <= 0) { ok = false; break; }
                t += (double)items[i].shape.width * items[i].shape.height * items[i].n_steps / vals[i].rate[fam];
            }
            if (ok && t < best_t) { best_t = t; c.fam = fam; }
        }
    }
    if (forced_fam >= 0) c.fam = forced_fam;
    if (const char *e = getenv("GEOCHAIN_PLAN_WGS_PER_CU")) c.wgs_per_cu = atoi(e);   // a measurement override
    for (size_t i = 0; i < items.size(); ++i) {
        int k = default_persistent_k(c.fam);
        if (all_tuned && vals[i].k[c.fam] > 0) k = vals[i].k[c.fam];
        if (forced_k > 0) k = forced_k;
        k = std::max(1, std::min(k, persistent_kmax(c.fam)));
        if (items[i].n_steps > 0 && items[i].n_steps < k) k = (int)items[i].n_steps;
        c.k.push_back(k);
    }
    return c;
}

__global__ void fill_u32_kernel(uint32_t *p, int64_t n, uint32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

static int plan_build(gc_dtype dtype, int op, const gc_item *items, int32_t n_items, gc_plan **out,
                      const PlanChoice *forced) {
    if (!out) return fail(GC_ERR_INVALID_ARG, "plan_out is NULL");
    *out = nullptr;
    if (elem_size(dtype) == 0) return fail(GC_ERR_INVALID_ARG, "unknown dtype %d", (int)dtype);
    if (op != OP_DILATE && op != OP_ERODE) return fail(GC_ERR_INVALID_ARG, "unknown op %d", op);
    if (n_items < 0 || (n_items > 0 && !items)) return fail(GC_ERR_INVALID_ARG, "bad item array");
    int mode = -1;
    for (int32_t i = 0; i < n_items; ++i) {
        const gc_item &it = items[i];
        int rc = validate_images(dtype, it.marker, it.mask, it.out, it.shape);
        if (rc != GC_OK) return fail(rc, "item %d: %s", i, g_last_error.c_str());
        if (it.n_steps < 0 && !it.mask)
            return fail(GC_ERR_UNSUPPORTED, "item %d: only geodesic items run to stability (n_steps < 0)", i);
        if (it.n_steps > INT32_MAX / 2) return fail(GC_ERR_UNSUPPORTED, "item %d: n_steps too large", i);
        const bool empty = it.shape.width == 0 || it.shape.height == 0;
        if (empty) continue;
        const int m = it.mask ? MODE_GEODESIC : MODE_PLAIN;
        if (mode >= 0 && m != mode)
            return fail(GC_ERR_UNSUPPORTED, "a plan is either all geodesic or all plain (item %d)", i);
        mode = m;
    }
    if (mode < 0) mode = MODE_GEODESIC;
    const size_t es = elem_size(dtype);

    gc_plan *p = new gc_plan();
    p->dtype = dtype;
    p->op = op;
    p->mode = mode;
    p->items.assign(items, items + n_items);
    if (hipGetDevice(&p->device) != hipSuccess) {
        (void)hipGetLastError();
        plan_free(p);
        return fail(GC_ERR_HIP, "hipGetDevice failed");
    }

    bool stab = false;
    for (const auto &it : p->items) stab = stab || (it.n_steps < 0 && it.shape.width > 0 && it.shape.height > 0);
    PlanChoice choice = forced ? *forced : choose_plan_batch(dtype, op, mode, p->items);
    if (stab) {
        // Run-to-stability plans keep the built-in launch shape: 128 x 128
        // regions, STAB_K steps per block (the change bits of a block are one
        // 32-bit word).
        choice.fam = FAM_128W;
        for (size_t i = 0; i < p->items.size(); ++i) {
            const int64_t ni = p->items[i].n_steps;
            choice.k[i] = ni > 0 && ni < STAB_K ? (int)ni : STAB_K;
        }
    }
    p->fam = choice.fam;
    const int side = region_side(p->fam);

    // ---- per-image descriptors, workspace layout, item list ----
    std::vector<PlanImage> imgs;
    std::vector<int> img_of_item;  // plan image index -> gc_item index
    size_t ws_bytes = 0;
    std::vector<size_t> ws_off;
    int64_t flags = 0;  // per-tile counters; at most the item count, checked below
    std::vector<std::pair<int, int>> copies;  // (gc_item index, kind) 0: n=0 copy, 1: marker->ws1
    for (int32_t i = 0; i < n_items; ++i) {
        const gc_item &it = p->items[i];
        if (it.shape.width == 0 || it.shape.height == 0) continue;
        if (it.n_steps == 0) { copies.push_back({i, 0}); continue; }
        PlanImage im{};
        im.marker = it.marker;
        im.mask = it.mask;
        im.out = it.out;
        im.pitch = it.shape.pitch;
        im.width = (int32_t)it.shape.width;
        im.height = (int32_t)it.shape.height;
        im.k = choice.k[i];
        // a run-to-stability image runs STAB_BLOCKS blocks per replay
        im.n_steps = it.n_steps < 0 ? STAB_BLOCKS * im.k : (int32_t)it.n_steps;
        im.core_x = side - 2 * im.k;
        im.core_y = side - 2 * im.k;
        im.tiles_x = (int32_t)((it.shape.width + im.core_x - 1) / im.core_x);
        im.tiles_y = (int32_t)((it.shape.height + im.core_y - 1) / im.core_y);
        im.blocks = (int32_t)((im.n_steps + im.k - 1) / im.k);
        im.active = 1;
        if (it.n_steps < 0) p->stab_imgs.push_back((int)imgs.size());
        im.flag_base = (int32_t)std::min<int64_t>(flags, INT32_MAX);
        flags += (int64_t)im.tiles_x * im.tiles_y;
        im.src0_ws1 = (it.out == it.marker && im.blocks == 1) ? 1 : 0;
        if (im.src0_ws1) copies.push_back({i, 1});
        const size_t bytes = (size_t)((it.shape.height - 1) * it.shape.pitch + it.shape.width) * es;
        const size_t aligned = (bytes + 255) & ~size_t(255);
        ws_off.push_back(ws_bytes);
        ws_bytes += 2 * aligned;
        imgs.push_back(im);
        img_of_item.push_back(i);
        if (it.n_steps > 0) p->px_steps += it.shape.width * it.shape.height * it.n_steps;
        p->max_k = std::max(p->max_k, im.k);
    }
    // items ordered by block, longest chains first within a block
    std::vector<int> order(imgs.size());
    for (size_t j = 0; j < order.size(); ++j) order[j] = (int)j;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return (int64_t)imgs[a].blocks * imgs[a].k > (int64_t)imgs[b].blocks * imgs[b].k;
    });
    int max_blocks = 0;
    for (auto &im : imgs) max_blocks = std::max(max_blocks, im.blocks);
    int64_t total_items = 0;
    for (auto &im : imgs) total_items += (int64_t)im.tiles_x * im.tiles_y * im.blocks;
    if (total_items > INT32_MAX) {
        plan_free(p);
        return fail(GC_ERR_UNSUPPORTED, "a plan of %lld work items (tiles x blocks) exceeds 2^31 - 1",
                    (long long)total_items);
    }
    std::vector<PlanItem> plan_items;
    plan_items.reserve((size_t)total_items);
    for (int b = 0; b < max_blocks; ++b)
        for (int j : order) {
            if (b >= imgs[j].blocks) continue;
            const int nt = imgs[j].tiles_x * imgs[j].tiles_y;
            for (int t = 0; t < nt; ++t) plan_items.push_back(PlanItem{j, t, b, 0});
        }
    p->n_items = (int32_t)plan_items.size();

    // ---- device allocations ----
    auto bail = [&](int rc) { plan_free(p); return rc; };
    // counters: [0] ticket, [1] error word, then one per tile, then STAB_BLOCKS
    // change words per run-to-stability image
    const int64_t n_change = (int64_t)p->stab_imgs.size() * STAB_BLOCKS;
    p->n_words = 2 + flags + n_change;
    if (hipMalloc((void **)&p->words_d, p->n_words * 4) != hipSuccess ||
        hipHostMalloc((void **)&p->error_h, 4, hipHostMallocDefault) != hipSuccess ||
        (n_change > 0 && hipHostMalloc((void **)&p->change_h, n_change * 4, hipHostMallocDefault) != hipSuccess)) {
        (void)hipGetLastError();
        return bail(fail(GC_ERR_NO_MEMORY, "plan counters"));
    }
    *p->error_h = 0;
    for (size_t q = 0; q < p->stab_imgs.size(); ++q)
        imgs[p->stab_imgs[q]].change = p->words_d + 2 + flags + (int64_t)q * STAB_BLOCKS;
    if (!imgs.empty()) {
        if (hipMalloc(&p->ws, ws_bytes) != hipSuccess) { (void)hipGetLastError(); return bail(fail(GC_ERR_NO_MEMORY, "plan workspace of %zu bytes", ws_bytes)); }
        for (size_t j = 0; j < imgs.size(); ++j) {
            const gc_item &it = p->items[img_of_item[j]];
            const size_t bytes = (size_t)((it.shape.height - 1) * it.shape.pitch + it.shape.width) * es;
            const size_t aligned = (bytes + 255) & ~size_t(255);
            imgs[j].ws0 = (char *)p->ws + ws_off[j];
            imgs[j].ws1 = (char *)p->ws + ws_off[j] + aligned;
        }
        if (hipMalloc((void **)&p->images_d, imgs.size() * sizeof(PlanImage)) != hipSuccess ||
            hipMalloc((void **)&p->items_d, std::max<size_t>(plan_items.size(), 1) * sizeof(PlanItem)) != hipSuccess) {
            (void)hipGetLastError();
            return bail(fail(GC_ERR_NO_MEMORY, "plan tables"));
        }
        if (hipMemcpy(p->images_d, imgs.data(), imgs.size() * sizeof(PlanImage), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(p->items_d, plan_items.data(), plan_items.size() * sizeof(PlanItem), hipMemcpyHostToDevice) != hipSuccess)
            return bail(fail(GC_ERR_HIP, "uploading plan tables"));
    }
    p->imgs_init = imgs;
    p->img_item = img_of_item;
    p->steps.assign(p->items.size(), -1);

    // ---- grid: as many workgroups as fit on the device at once ----
    const PersistentFns fns = persistent_fns(dtype, op, mode, p->fam, n_change > 0);
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fns.kernel, fns.threads, 0) != hipSuccess)
        return bail(fail(GC_ERR_HIP, "occupancy query failed"));
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess)
        return bail(fail(GC_ERR_HIP, "CU count query failed"));
    if (choice.wgs_per_cu > 0) per_cu = std::min(per_cu, choice.wgs_per_cu);
    p->grid = (int32_t)std::max<int64_t>(1, std::min<int64_t>((int64_t)std::max(per_cu, 1) * cus,
                                                               std::max<int32_t>(p->n_items, 1)));
    // Tests of the dealing: GEOCHAIN_PLAN_GRID=<n> gives plans built while
    // it is set a grid of n workgroups, whether or not they fit on the
    // device at once (items are drawn in list order, so any grid finishes).
    if (const char *e = getenv("GEOCHAIN_PLAN_GRID")) {
        const long v = strtol(e, nullptr, 10);
        if (v > 0 && v <= (1L << 20)) p->grid = (int32_t)v;
    }

    // ---- record the launch ----
    if (hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking) != hipSuccess)
        return bail(fail(GC_ERR_HIP, "stream creation failed"));
    if (hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return bail(fail(GC_ERR_HIP, "graph capture failed to start"));
    bool cap_ok = true;
    // Counters start at zero: a fill kernel, not a memset node.
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)std::min<int64_t>((p->n_words + 255) / 256, 1024)), dim3(256), 0,
                       p->cap_stream, p->words_d, p->n_words, 0u);
    cap_ok = cap_ok && hipGetLastError() == hipSuccess;
    for (auto &c : copies) {
        const gc_item &it = p->items[c.first];
        void *dst = it.out;
        if (c.second == 1) {
            for (size_t j = 0; j < imgs.size(); ++j)
                if (img_of_item[j] == c.first) dst = imgs[j].ws1;
        }
        if (dst != it.marker)
            cap_ok = cap_ok && hipMemcpy2DAsync(dst, it.shape.pitch * es, it.marker, it.shape.pitch * es,
                                                it.shape.width * es, it.shape.height, hipMemcpyDeviceToDevice,
                                                p->cap_stream) == hipSuccess;
    }
    if (p->n_items > 0) {
        PersistentArgs a{};
        a.images = p->images_d;
        a.items = p->items_d;
        a.n_items = p->n_items;
        a.ticket = p->words_d;
        a.error = p->words_d + 1;
        a.flags = p->words_d + 2;
        a.wait_ticks = PLAN_WAIT_TICKS;
        // Tests of the error path: GEOCHAIN_PLAN_WAIT_TICKS=<n> bounds the
        // waits of plans built while it is set to n ticks (0: they fail at once).
        if (const char *e = getenv("GEOCHAIN_PLAN_WAIT_TICKS")) a.wait_ticks = strtoull(e, nullptr, 10);
        // Consecutive items per ticket (neighbouring tiles of one image, run
        // by one workgroup back to back, share its XCD's L2): about eight
        // tickets per workgroup, at most 4 items each.  Measured on the
        // 64-image batch (3.9e5 items, 512 workgroups): 28.7 ms with 1 item
        // per ticket, 24.7 with 2, 22.0 with 4, 22.3 with 8, 26.6 with 16;
        // a 16-image run-to-stability replay (1e4 items) is fastest with 2.
        a.chunk = (int32_t)std::max<int64_t>(1, std::min<int64_t>(4, p->n_items / ((int64_t)p->grid * 8)));
        fns.launch(a, p->grid, p->cap_stream);
        cap_ok = cap_ok && hipGetLastError() == hipSuccess;
        // Error word to pinned host memory for gc_plan_status.
        cap_ok = cap_ok && hipMemcpyAsync(p->error_h, p->words_d + 1, 4, hipMemcpyDeviceToHost, p->cap_stream) == hipSuccess;
        if (n_change > 0)
            cap_ok = cap_ok && hipMemcpyAsync(p->change_h, p->words_d + 2 + flags, n_change * 4, hipMemcpyDeviceToHost,
                                              p->cap_stream) == hipSuccess;
    }
    hipError_t ec = hipStreamEndCapture(p->cap_stream, &p->graph);
    if (ec != hipSuccess || !cap_ok) return bail(fail(GC_ERR_HIP, "graph capture failed: %s", hipGetErrorString(ec)));
    if (hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0) != hipSuccess)
        return bail(fail(GC_ERR_HIP, "graph instantiation failed"));
    *out = p;
    return GC_OK;
}

static int plan_time(gc_plan *p, int reps, double *ms_out) {
    hipStream_t st = p->cap_stream;
    hipEvent_t a = nullptr, b = nullptr;
    float ms = 0;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e == hipSuccess) e = hipGraphLaunch(p->exec, st);  // warm-up
    if (e == hipSuccess) e = hipEventRecord(a, st);
    for (int i = 0; i < reps && e == hipSuccess; ++i) e = hipGraphLaunch(p->exec, st);
    if (e == hipSuccess) e = hipEventRecord(b, st);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (e != hipSuccess) return fail(GC_ERR_HIP, "timing a plan failed: %s", hipGetErrorString(e));
    *ms_out = ms / reps;
    return *p->error_h ? fail(GC_ERR_HIP, "dependency wait hit its bound while tuning") : GC_OK;
}

static int autotune(gc_dtype dtype, int op, int geodesic, int64_t width, int64_t height, TuneVal *out) {
    const size_t es = elem_size(dtype);
    // Enough copies of the size class to fill the device, as in a batch.
    const int64_t px = std::max<int64_t>(width * height, 1);
    const int copies = (int)std::max<int64_t>(1, std::min<int64_t>(64, (2048LL * 2048LL + px - 1) / px));
    const size_t bytes = (size_t)(width * height) * es;
    void *buf = nullptr;
    if (hipMalloc(&buf, std::max<size_t>(bytes, 1) * 3 * copies) != hipSuccess) {
        (void)hipGetLastError();
        return fail(GC_ERR_NO_MEMORY, "autotune scratch");
    }
    if (hipMemset(buf, 0, std::max<size_t>(bytes, 1) * 3 * copies) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(buf);
        return fail(GC_ERR_HIP, "autotune scratch clear failed");
    }
    const int n_steps = 240;
    TuneVal tv;
    double best_rate = 0;
    for (int fam = 0; fam < NUM_FAMS; ++fam) {
        for (int k = 4; k <= persistent_kmax(fam); k += 4) {
            std::vector<gc_item> items(copies);
            for (int c = 0; c < copies; ++c) {
                char *base = (char *)buf + (size_t)c * 3 * bytes;
                items[c].marker = base;
                items[c].mask = geodesic ? base + bytes : nullptr;
                items[c].out = base + 2 * bytes;
                items[c].shape = gc_shape{width, height, width};
                items[c].n_steps = n_steps;
            }
            PlanChoice ch;
            ch.fam = fam;
            ch.k.assign(copies, k);
            gc_plan *p = nullptr;
            int rc = plan_build(dtype, op, items.data(), copies, &p, &ch);
            if (rc != GC_OK) { (void)hipFree(buf); return rc; }
            double ms = 0;
            rc = plan_time(p, 3, &ms);
            plan_free(p);
            if (rc != GC_OK) { (void)hipFree(buf); return rc; }
            const double rate = (double)px * copies * n_steps / (ms * 1e-3);
            if (rate > tv.rate[fam]) { tv.rate[fam] = rate; tv.k[fam] = k; }
            if (rate > best_rate) { best_rate = rate; tv.best_fam = fam; }
        }
    }
    (void)hipFree(buf);
    *out = tv;
    return GC_OK;
}

// ---------------------------------------------------------------------------
// differentiation: per-step codes and the reverse gather
// ---------------------------------------------------------------------------
static int validate_batch(gc_dtype dtype, const gc_shape &s, int32_t n_images, int64_t image_stride,
                          int64_t n_steps) {
    int rc = validate_shape(dtype, s);
    if (rc != GC_OK) return rc;
    if (dtype != GC_F32 && dtype != GC_F64) return fail(GC_ERR_UNSUPPORTED, "gradients need f32 or f64 images");
    if (n_images < 0) return fail(GC_ERR_INVALID_ARG, "n_images < 0");
    if (n_steps < 0) return fail(GC_ERR_INVALID_ARG, "n_steps < 0");
    if (n_images > 65535) return fail(GC_ERR_UNSUPPORTED, "at most 65535 images per call");
    // the gradient kernels take one row of workgroups per core height
    const int64_t cy = dtype == GC_F32 ? GradTile<float>::CY : GradTile<double>::CY;
    if ((s.height + cy - 1) / cy > 65535)
        return fail(GC_ERR_UNSUPPORTED, "gradients take images of at most %lld rows", (long long)(65535 * cy));
    const int64_t span = s.height > 0 ? (s.height - 1) * s.pitch + s.width : 0;
    if (n_images > 1 && image_stride < span)
        return fail(GC_ERR_INVALID_ARG, "image_stride %lld < image span %lld", (long long)image_stride,
                    (long long)span);
    return GC_OK;
}

// Byte extent of a batch of images.
static std::pair<uintptr_t, uintptr_t> batch_extent(const void *p, const gc_shape &s, int32_t n, int64_t stride,
                                                     size_t es) {
    uintptr_t lo = (uintptr_t)p;
    if (s.width == 0 || s.height == 0 || n == 0) return {lo, lo};
    const uint64_t span = (uint64_t)(s.height - 1) * s.pitch + s.width;
    return {lo, lo + ((uint64_t)(n - 1) * stride + span) * es};
}

template <typename T>
static dim3 block_grid(const gc_shape &s, int32_t n_images) {
    constexpr int CY = GradTile<T>::CY;
    return dim3((unsigned)((s.width + GB_CX - 1) / GB_CX), (unsigned)((s.height + CY - 1) / CY), (unsigned)n_images);
}

template <typename T>
static void launch_codes(int op, const GradBlockArgs &a, const gc_shape &s, int32_t n, hipStream_t st) {
    const dim3 grid = block_grid<T>(s, n), block(GradTile<T>::THREADS);
    if (op == OP_DILATE)
        hipLaunchKernelGGL((block_codes_kernel<T, OP_DILATE>), grid, block, 0, st, a);
    else
        hipLaunchKernelGGL((block_codes_kernel<T, OP_ERODE>), grid, block, 0, st, a);
}

template <typename T>
static void launch_bwd(const GradBlockArgs &a, const gc_shape &s, int32_t n, hipStream_t st) {
    hipLaunchKernelGGL((block_bwd_kernel<T>), block_grid<T>(s, n), dim3(GradTile<T>::THREADS), 0, st, a);
}

// Forward with codes: blocks of up to GB_K steps per launch, ping-pong
// through the workspace, the last block writing out.
static int run_fwd_codes(gc_dtype dtype, int op, const void *marker, const void *mask, void *out, uint8_t *codes,
                         const gc_shape &s, int32_t n, int64_t stride, int64_t n_steps, hipStream_t st) {
    const size_t es = elem_size(dtype);
    if (s.width == 0 || s.height == 0 || n == 0) return GC_OK;
    const int64_t span = (s.height - 1) * s.pitch + s.width;
    const int64_t istride = n > 1 ? stride : span;
    const size_t batch_bytes = (size_t)((int64_t)(n - 1) * istride + span) * es;
    if (n_steps == 0) {
        if (out != marker)
            GC_HIP(hipMemcpyAsync(out, marker, batch_bytes, hipMemcpyDeviceToDevice, st));
        return GC_OK;
    }
    const size_t half = (batch_bytes + 255) & ~size_t(255);
    Workspace *ws = nullptr;
    int rc = get_workspace(st, 2 * half, 0, &ws);
    if (rc != GC_OK) return rc;
    void *w[2] = {ws->buf, (char *)ws->buf + half};
    const int64_t blocks = (n_steps + GB_K - 1) / GB_K;
    const void *cur = marker;
    if (out == marker && blocks == 1) {
        GC_HIP(hipMemcpyAsync(w[1], marker, batch_bytes, hipMemcpyDeviceToDevice, st));
        cur = w[1];
    }
    const int64_t codes_step = s.height * s.width;
    for (int64_t b = 0; b < blocks; ++b) {
        const int64_t t0 = b * GB_K;
        const int kb = (int)std::min<int64_t>(GB_K, n_steps - t0);
        void *dst = b == blocks - 1 ? out : w[b & 1];
        GradBlockArgs a{};
        a.src = cur;
        a.mask = mask;
        a.dst = dst;
        a.codes = codes + t0 * codes_step;
        a.codes_step = codes_step;
        a.codes_image = n_steps * codes_step;
        a.image_stride = istride;
        a.pitch = s.pitch;
        a.width = (int32_t)s.width;
        a.height = (int32_t)s.height;
        a.k = kb;
        const int pr = prof_begin(st, kb);
        if (dtype == GC_F32) launch_codes<float>(op, a, s, n, st);
        else launch_codes<double>(op, a, s, n, st);
        prof_end(pr, st);
        GC_HIP(hipGetLastError());
        cur = dst;
    }
    return GC_OK;
}

// Reverse pass: the same blocks from last to first.
static int run_bwd(gc_dtype dtype, const uint8_t *codes, const void *g_out, void *g_marker, void *g_mask,
                   const gc_shape &s, int32_t n, int64_t stride, int64_t n_steps, hipStream_t st) {
    const size_t es = elem_size(dtype);
    if (s.width == 0 || s.height == 0 || n == 0) return GC_OK;
    const int64_t span = (s.height - 1) * s.pitch + s.width;
    const int64_t istride = n > 1 ? stride : span;
    const size_t batch_bytes = (size_t)((int64_t)(n - 1) * istride + span) * es;
    if (n_steps == 0) {
        GC_HIP(hipMemcpyAsync(g_marker, g_out, batch_bytes, hipMemcpyDeviceToDevice, st));
        return GC_OK;
    }
    const size_t half = (batch_bytes + 255) & ~size_t(255);
    Workspace *ws = nullptr;
    int rc = get_workspace(st, 2 * half, 0, &ws);
    if (rc != GC_OK) return rc;
    void *w[2] = {ws->buf, (char *)ws->buf + half};
    const int64_t codes_step = s.height * s.width;
    const int64_t blocks = (n_steps + GB_K - 1) / GB_K;
    const void *cur = g_out;
    for (int64_t b = blocks - 1; b >= 0; --b) {
        const int64_t t0 = b * GB_K;
        const int kb = (int)std::min<int64_t>(GB_K, n_steps - t0);
        void *dst = b == 0 ? g_marker : w[b & 1];
        GradBlockArgs a{};
        a.src = cur;
        a.dst = dst;
        a.g_mask = g_mask;
        a.codes = const_cast<uint8_t *>(codes) + t0 * codes_step;
        a.codes_step = codes_step;
        a.codes_image = n_steps * codes_step;
        a.image_stride = istride;
        a.pitch = s.pitch;
        a.width = (int32_t)s.width;
        a.height = (int32_t)s.height;
        a.k = kb;
        const int pr = prof_begin(st, kb);
        if (dtype == GC_F32) launch_bwd<float>(a, s, n, st);
        else launch_bwd<double>(a, s, n, st);
        prof_end(pr, st);
        GC_HIP(hipGetLastError());
        cur = dst;
    }
    return GC_OK;
}

// Forward with source ids: blocks of up to GB_K steps per launch; values
// ping-pong through the workspace as in run_fwd_codes, ids likewise through
// two id planes, the last block writing out and sources.
template <typename T>
static void launch_src(int op, const SrcBlockArgs &a, const gc_shape &s, int32_t n, hipStream_t st) {
    const dim3 grid = block_grid<T>(s, n), block(GradTile<T>::THREADS);
    if (op == OP_DILATE)
        hipLaunchKernelGGL((block_src_kernel<T, OP_DILATE>), grid, block, 0, st, a);
    else
        hipLaunchKernelGGL((block_src_kernel<T, OP_ERODE>), grid, block, 0, st, a);
}

static int run_fwd_sources(gc_dtype dtype, int op, const void *marker, const void *mask, void *out,
                           uint32_t *sources, const gc_shape &s, int32_t n, int64_t stride, int64_t n_steps,
                           hipStream_t st) {
    const size_t es = elem_size(dtype);
    if (s.width == 0 || s.height == 0 || n == 0) return GC_OK;
    const int64_t span = (s.height - 1) * s.pitch + s.width;
    const int64_t istride = n > 1 ? stride : span;
    const int64_t batch_elems = (int64_t)(n - 1) * istride + span;
    const size_t half = ((size_t)batch_elems * es + 255) & ~size_t(255);
    const size_t ihalf = ((size_t)batch_elems * 4 + 255) & ~size_t(255);
    const int64_t blocks = std::max<int64_t>(1, (n_steps + GB_K - 1) / GB_K);
    Workspace *ws = nullptr;
    int rc = get_workspace(st, 2 * half + (blocks > 1 ? 2 * ihalf : 0), 0, &ws);
    if (rc != GC_OK) return rc;
    void *w[2] = {ws->buf, (char *)ws->buf + half};
    uint32_t *iw[2] = {(uint32_t *)((char *)ws->buf + 2 * half), (uint32_t *)((char *)ws->buf + 2 * half + ihalf)};
    const void *cur = marker;
    if (out == marker && blocks == 1) {
        GC_HIP(hipMemcpyAsync(w[1], marker, (size_t)batch_elems * es, hipMemcpyDeviceToDevice, st));
        cur = w[1];
    }
    const uint32_t *ids = nullptr;
    for (int64_t b = 0; b < blocks; ++b) {
        const int kb = (int)std::min<int64_t>(GB_K, n_steps - b * GB_K);   // 0 for a zero-step chain
        const bool last = b == blocks - 1;
        SrcBlockArgs a{};
        a.src = cur;
        a.mask = mask;
        a.dst = last ? out : w[b & 1];
        a.ids_in = ids;
        a.ids_out = last ? sources : iw[b & 1];
        a.image_stride = istride;
        a.pitch = s.pitch;
        a.width = (int32_t)s.width;
        a.height = (int32_t)s.height;
        a.k = kb;
        const int pr = prof_begin(st, kb);
        if (dtype == GC_F32) launch_src<float>(op, a, s, n, st);
        else launch_src<double>(op, a, s, n, st);
        prof_end(pr, st);
        GC_HIP(hipGetLastError());
        cur = a.dst;
        ids = a.ids_out;
    }
    return GC_OK;
}

// Reverse pass from source ids: the own-pixel pass (which also sets every
// other marker-gradient pixel to zero), then the atomic pass.
static int run_bwd_sources(gc_dtype dtype, const uint32_t *sources, const void *g_out, void *g_marker,
                           void *g_mask, const gc_shape &s, int32_t n, int64_t stride, hipStream_t st) {
    if (s.width == 0 || s.height == 0 || n == 0) return GC_OK;
    const int64_t span = (s.height - 1) * s.pitch + s.width;
    const int64_t istride = n > 1 ? stride : span;
    // x: columns in groups of 256; y: rows (one per block up to 65535, then
    // strided); z: images
    const dim3 grid((unsigned)((s.width + 255) / 256), (unsigned)std::min<int64_t>(s.height, 65535), (unsigned)n);
    SrcScatterArgs a{};
    a.ids = sources;
    a.g_out = g_out;
    a.g_marker = g_marker;
    a.g_mask = g_mask;
    a.image_stride = istride;
    a.pitch = s.pitch;
    a.width = (int32_t)s.width;
    a.height = (int32_t)s.height;
    a.n_images = n;
    a.span = (uint32_t)span;
    if (dtype == GC_F32) {
        hipLaunchKernelGGL(src_local_kernel<float>, grid, dim3(256), 0, st, a);
        hipLaunchKernelGGL(src_scatter_kernel<float>, grid, dim3(256), 0, st, a);
    } else {
        hipLaunchKernelGGL(src_local_kernel<double>, grid, dim3(256), 0, st, a);
        hipLaunchKernelGGL(src_scatter_kernel<double>, grid, dim3(256), 0, st, a);
    }
    GC_HIP(hipGetLastError());
    return GC_OK;
}

}  // namespace geochain

using namespace geochain;

// Enum arguments arrive from C callers, where any int is a valid value of
// the type; in C++ reading an out-of-range value through the enum type is
// undefined.  Entry points therefore look at the bits first (through
// memcpy, which reads no enum) and refuse unknown values before the
// argument is used.
template <typename E>
static int enum_bits(const E *e) {
    static_assert(sizeof(E) == sizeof(int), "C enums are int-sized here");
    int v;
    memcpy(&v, e, sizeof v);
    return v;
}

#define GC_CHECK_DTYPE(d)                                                                   \
    do {                                                                                    \
        const int v_ = enum_bits(&(d));                                                     \
        if (v_ != GC_U8 && v_ != GC_F32 && v_ != GC_F64) {                                  \
            g_last_error.clear();                                                           \
            return fail(GC_ERR_INVALID_ARG, "unknown dtype %d", v_);                        \
        }                                                                                   \
    } while (0)
#define GC_CHECK_OP(o)                                                                      \
    do {                                                                                    \
        const int v_ = enum_bits(&(o));                                                     \
        if (v_ != GC_DILATE && v_ != GC_ERODE) {                                            \
            g_last_error.clear();                                                           \
            return fail(GC_ERR_INVALID_ARG, "unknown op %d", v_);                           \
        }                                                                                   \
    } while (0)


template <typename T>
static int run_value_scan_t(const T *img, const gc_shape &s, uint32_t *found, void *stream) {
    hipStream_t st = (hipStream_t)stream;
    Workspace *ws = nullptr;
    int rc = get_workspace(stream, 0, 1, &ws);
    if (rc != GC_OK) return rc;
    const bool vec = rows_aligned16(s, sizeof(T), img, img);
    const PixelArgs<T> p = pixel_args<T>(s, img, nullptr, nullptr, vec);
    hipLaunchKernelGGL(fill_words_kernel, dim3(1), dim3(128), 0, st, ws->words, 1, 0u);
    const int grid = px_grid(p.n_chunks, 4096);
    if (vec)
        hipLaunchKernelGGL((value_scan_kernel<T, true>), dim3(grid), dim3(PX_THREADS), 0, st, p, ws->words);
    else
        hipLaunchKernelGGL((value_scan_kernel<T, false>), dim3(grid), dim3(PX_THREADS), 0, st, p, ws->words);
    GC_HIP(hipGetLastError());
    {
        const int wrc = read_words(ws, 1, st);
        if (wrc != GC_OK) return wrc;
    }
    *found = ws->host_words[0];
    return GC_OK;
}

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
    GC_CHECK_DTYPE(dtype);
    return geodesic_chain(dtype, OP_DILATE, marker, mask, out, shape, n_steps, hip_stream);
}

int gc_geodesic_erode_chain(gc_dtype dtype, const void *marker, const void *mask, void *out,
                            gc_shape shape, int64_t n_steps, void *hip_stream) {
    GC_CHECK_DTYPE(dtype);
    return geodesic_chain(dtype, OP_ERODE, marker, mask, out, shape, n_steps, hip_stream);
}

int gc_geodesic_chain_noalloc(gc_dtype dtype, gc_op op, const void *marker, const void *mask, void *out,
                              gc_shape shape, int64_t n_steps, void *hip_stream) {
    GC_CHECK_DTYPE(dtype);
    GC_CHECK_OP(op);
    g_last_error.clear();
    int rc = validate_images(dtype, marker, mask, out, shape);
    if (rc != GC_OK) return rc;
    if (!(shape.width == 0 || shape.height == 0) && !mask) return fail(GC_ERR_INVALID_ARG, "null mask");
    if (n_steps < 0) return fail(GC_ERR_INVALID_ARG, "n_steps < 0");
    if (shape.width == 0 || shape.height == 0) return GC_OK;
    // the size check comes before any HIP call
    const size_t bytes = (size_t)((shape.height - 1) * shape.pitch + shape.width) * elem_size(dtype);
    if (bytes > NOALLOC_SCRATCH_BYTES)
        return fail(GC_ERR_UNSUPPORTED, "image spans %zu bytes; the no-allocation chain holds at most %zu",
                    bytes, NOALLOC_SCRATCH_BYTES);
    void *work = nullptr;
    rc = scratch_address(&work);
    if (rc != GC_OK) return rc;
    return run_chain(dtype, enum_bits(&op), MODE_GEODESIC, marker, mask, out, shape, n_steps, hip_stream, work,
                     NOALLOC_SCRATCH_BYTES);
}

int gc_geodesic_chain_batch(gc_dtype dtype, gc_op op, const void *marker, const void *mask, void *out,
                            gc_shape shape, int32_t n_images, int64_t image_stride, int64_t n_steps,
                            void *hip_stream) {
    GC_CHECK_DTYPE(dtype);
    GC_CHECK_OP(op);
    g_last_error.clear();
    int rc = validate_shape(dtype, shape);
    if (rc != GC_OK) return rc;
    if (n_images < 0) return fail(GC_ERR_INVALID_ARG, "n_images < 0");
    if (n_images > 65535) return fail(GC_ERR_UNSUPPORTED, "at most 65535 images per call");
    if (n_steps < 0) return fail(GC_ERR_INVALID_ARG, "n_steps < 0");
    const bool empty = shape.width == 0 || shape.height == 0 || n_images == 0;
    if (empty) return GC_OK;
    const int64_t span = (shape.height - 1) * shape.pitch + shape.width;
    if (n_images > 1 && image_stride < span)
        return fail(GC_ERR_INVALID_ARG, "image_stride %lld < image span %lld", (long long)image_stride,
                    (long long)span);
    if (!marker || !mask || !out) return fail(GC_ERR_INVALID_ARG, "null pointer");
    const size_t es = elem_size(dtype);
    const auto eo = batch_extent(out, shape, n_images, image_stride, es);
    if (overlap(eo, batch_extent(mask, shape, n_images, image_stride, es)))
        return fail(GC_ERR_ALIAS, "out overlaps mask");
    if (out != marker && overlap(eo, batch_extent(marker, shape, n_images, image_stride, es)))
        return fail(GC_ERR_ALIAS, "out partially overlaps marker");
    return run_chain(dtype, enum_bits(&op), MODE_GEODESIC, marker, mask, out, shape, n_steps, hip_stream, nullptr, 0,
                     n_images, image_stride);
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
    GC_CHECK_DTYPE(dtype);
    return plain_chain(dtype, OP_DILATE, in, out, shape, n_steps, hip_stream);
}

int gc_erode_chain(gc_dtype dtype, const void *in, void *out, gc_shape shape, int64_t n_steps,
                   void *hip_stream) {
    GC_CHECK_DTYPE(dtype);
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
    GC_CHECK_DTYPE(dtype);
    return reconstruct(dtype, OP_DILATE, marker, mask, out, shape, max_steps, steps_out, hip_stream);
}

int gc_reconstruct_by_erosion(gc_dtype dtype, const void *marker, const void *mask, void *out,
                              gc_shape shape, int64_t max_steps, int64_t *steps_out,
                              void *hip_stream) {
    GC_CHECK_DTYPE(dtype);
    return reconstruct(dtype, OP_ERODE, marker, mask, out, shape, max_steps, steps_out, hip_stream);
}

static int geodesic_operator(gc_dtype dtype, int which, const void *f, void *out, gc_shape shape, double h,
                             int64_t size, int64_t max_steps, int64_t *steps_out, void *stream) {
    g_last_error.clear();
    if (steps_out) *steps_out = 0;
    int rc = validate_shape(dtype, shape);
    if (rc != GC_OK) return rc;
    const bool empty = shape.width == 0 || shape.height == 0;
    if (!empty && (!f || !out)) return fail(GC_ERR_INVALID_ARG, "null image pointer");
    const size_t es = elem_size(dtype);
    if (!empty && overlap(extent(out, shape, es), extent(f, shape, es)))
        return fail(GC_ERR_ALIAS, "out overlaps f (f is the mask of the reconstruction)");
    if (which == GOP_HMAX || which == GOP_DOME) {
        if (!finite_bits(h) || h < 0) return fail(GC_ERR_INVALID_ARG, "h must be finite and >= 0");
        if (dtype == GC_U8 && h != std::floor(h))
            return fail(GC_ERR_INVALID_ARG, "h must be an integer for u8 images");
    }
    if (which == GOP_OPEN_REC && size < 0) return fail(GC_ERR_INVALID_ARG, "size < 0");
    if (empty) return GC_OK;
    switch (dtype) {
        case GC_U8:
            return run_operator_t<uint8_t>(dtype, which, (const uint8_t *)f, (uint8_t *)out, shape,
                                           (uint8_t)std::min(h, 255.0), size, max_steps, steps_out, stream);
        case GC_F32:
            return run_operator_t<float>(dtype, which, (const float *)f, (float *)out, shape, (float)h, size,
                                         max_steps, steps_out, stream);
        case GC_F64:
            return run_operator_t<double>(dtype, which, (const double *)f, (double *)out, shape, h, size,
                                          max_steps, steps_out, stream);
    }
    return fail(GC_ERR_INVALID_ARG, "unknown dtype");
}

int gc_hmax(gc_dtype dtype, const void *f, void *out, gc_shape shape, double h, int64_t max_steps,
            int64_t *steps_out, void *hip_stream) {
    GC_CHECK_DTYPE(dtype);
    return geodesic_operator(dtype, GOP_HMAX, f, out, shape, h, 0, max_steps, steps_out, hip_stream);
}

int gc_dome(gc_dtype dtype, const void *f, void *out, gc_shape shape, double h, int64_t max_steps,
            int64_t *steps_out, void *hip_stream) {
    GC_CHECK_DTYPE(dtype);
    return geodesic_operator(dtype, GOP_DOME, f, out, shape, h, 0, max_steps, steps_out, hip_stream);
}

int gc_hfill(gc_dtype dtype, const void *f, void *out, gc_shape shape, int64_t max_steps,
             int64_t *steps_out, void *hip_stream) {
    GC_CHECK_DTYPE(dtype);
    return geodesic_operator(dtype, GOP_HFILL, f, out, shape, 0.0, 0, max_steps, steps_out, hip_stream);
}

int gc_raobj(gc_dtype dtype, const void *f, void *out, gc_shape shape, int64_t max_steps,
             int64_t *steps_out, void *hip_stream) {
    GC_CHECK_DTYPE(dtype);
    return geodesic_operator(dtype, GOP_RAOBJ, f, out, shape, 0.0, 0, max_steps, steps_out, hip_stream);
}

int gc_open_by_reconstruction(gc_dtype dtype, const void *f, void *out, gc_shape shape, int64_t size,
                              int64_t max_steps, int64_t *steps_out, void *hip_stream) {
    GC_CHECK_DTYPE(dtype);
    return geodesic_operator(dtype, GOP_OPEN_REC, f, out, shape, 0.0, size, max_steps, steps_out,
                             hip_stream);
}

int gc_granulometry(gc_dtype dtype, const void *f, gc_shape shape, int32_t s_max, double *G, double *PS,
                    void *hip_stream) {
    GC_CHECK_DTYPE(dtype);
    g_last_error.clear();
    int rc = validate_shape(dtype, shape);
    if (rc != GC_OK) return rc;
    if (s_max < 0) return fail(GC_ERR_INVALID_ARG, "s_max < 0");
    if (!G) return fail(GC_ERR_INVALID_ARG, "null G");
    if (shape.width == 0 || shape.height == 0) {
        std::fill(G, G + s_max + 1, 0.0);
    } else {
        if (!f) return fail(GC_ERR_INVALID_ARG, "null image pointer");
        switch (dtype) {
            case GC_U8: rc = run_granulometry_t<uint8_t>(dtype, (const uint8_t *)f, shape, s_max, G, hip_stream); break;
            case GC_F32: rc = run_granulometry_t<float>(dtype, (const float *)f, shape, s_max, G, hip_stream); break;
            case GC_F64: rc = run_granulometry_t<double>(dtype, (const double *)f, shape, s_max, G, hip_stream); break;
        }
        if (rc != GC_OK) return rc;
    }
    if (PS)
        for (int i = 0; i < s_max; ++i) PS[i] = G[i] - G[i + 1];
    return GC_OK;
}

int gc_asf(gc_dtype dtype, const void *f, void *out, gc_shape shape, int32_t s_max, void *hip_stream) {
    GC_CHECK_DTYPE(dtype);
    g_last_error.clear();
    int rc = validate_images(dtype, f, nullptr, out, shape);
    if (rc != GC_OK) return rc;
    if (s_max < 0) return fail(GC_ERR_INVALID_ARG, "s_max < 0");
    if (shape.width == 0 || shape.height == 0) return GC_OK;
    return run_asf(dtype, f, out, shape, s_max, hip_stream);
}

int gc_quasi_distance(gc_dtype dtype, const void *f, int32_t *dist, void *residual, gc_shape shape,
                      int32_t lipschitz, int64_t *erosion_steps, int64_t *eta_steps, void *hip_stream) {
    GC_CHECK_DTYPE(dtype);
    g_last_error.clear();
    if (erosion_steps) *erosion_steps = 0;
    if (eta_steps) *eta_steps = 0;
    int rc = validate_shape(dtype, shape);
    if (rc != GC_OK) return rc;
    if (shape.width == 0 || shape.height == 0) return GC_OK;
    if (!f || !dist) return fail(GC_ERR_INVALID_ARG, "null image pointer");
    if ((uintptr_t)dist % 4) return fail(GC_ERR_INVALID_ARG, "dist must be 4-byte aligned");
    const size_t es = elem_size(dtype);
    const auto ef = extent(f, shape, es);
    const auto ed = extent(dist, shape, 4);
    if (overlap(ef, ed)) return fail(GC_ERR_ALIAS, "dist overlaps f");
    if (residual) {
        const auto er = extent(residual, shape, es);
        if (overlap(er, ef) || overlap(er, ed)) return fail(GC_ERR_ALIAS, "residual overlaps f or dist");
    }
    switch (dtype) {
        case GC_U8:
            return run_qdt_t<uint8_t>((const uint8_t *)f, dist, (uint8_t *)residual, shape, lipschitz != 0,
                                      erosion_steps, eta_steps, hip_stream);
        case GC_F32:
            return run_qdt_t<float>((const float *)f, dist, (float *)residual, shape, lipschitz != 0,
                                    erosion_steps, eta_steps, hip_stream);
        case GC_F64:
            return run_qdt_t<double>((const double *)f, dist, (double *)residual, shape, lipschitz != 0,
                                     erosion_steps, eta_steps, hip_stream);
    }
    return fail(GC_ERR_INVALID_ARG, "unknown dtype");
}

int gc_geodesic_chain_fwd_codes(gc_dtype dtype, gc_op op, const void *marker, const void *mask, void *out,
                                uint8_t *codes, gc_shape shape, int32_t n_images, int64_t image_stride,
                                int64_t n_steps, void *hip_stream) {
    GC_CHECK_DTYPE(dtype);
    GC_CHECK_OP(op);
    g_last_error.clear();
    int rc = validate_batch(dtype, shape, n_images, image_stride, n_steps);
    if (rc != GC_OK) return rc;
    if (op != GC_DILATE && op != GC_ERODE) return fail(GC_ERR_INVALID_ARG, "unknown op");
    const bool empty = shape.width == 0 || shape.height == 0 || n_images == 0;
    if (empty) return GC_OK;
    if (!marker || !mask || !out || (n_steps > 0 && !codes)) return fail(GC_ERR_INVALID_ARG, "null pointer");
    const size_t es = elem_size(dtype);
    const auto eo = batch_extent(out, shape, n_images, image_stride, es);
    if (overlap(eo, batch_extent(mask, shape, n_images, image_stride, es)))
        return fail(GC_ERR_ALIAS, "out overlaps mask");
    if (out != marker && overlap(eo, batch_extent(marker, shape, n_images, image_stride, es)))
        return fail(GC_ERR_ALIAS, "out partially overlaps marker");
    return run_fwd_codes(dtype, (int)op, marker, mask, out, codes, shape, n_images, image_stride, n_steps,
                         (hipStream_t)hip_stream);
}

int gc_geodesic_chain_bwd(gc_dtype dtype, gc_op op, const uint8_t *codes, const void *grad_out,
                          void *grad_marker, void *grad_mask, gc_shape shape, int32_t n_images,
                          int64_t image_stride, int64_t n_steps, void *hip_stream) {
    GC_CHECK_DTYPE(dtype);
    GC_CHECK_OP(op);
    g_last_error.clear();
    int rc = validate_batch(dtype, shape, n_images, image_stride, n_steps);
    if (rc != GC_OK) return rc;
    if (op != GC_DILATE && op != GC_ERODE) return fail(GC_ERR_INVALID_ARG, "unknown op");
    const bool empty = shape.width == 0 || shape.height == 0 || n_images == 0;
    if (empty) return GC_OK;
    if (!grad_out || !grad_marker || !grad_mask || (n_steps > 0 && !codes))
        return fail(GC_ERR_INVALID_ARG, "null pointer");
    const size_t es = elem_size(dtype);
    const auto egm = batch_extent(grad_marker, shape, n_images, image_stride, es);
    if (overlap(egm, batch_extent(grad_out, shape, n_images, image_stride, es)) ||
        overlap(egm, batch_extent(grad_mask, shape, n_images, image_stride, es)))
        return fail(GC_ERR_ALIAS, "grad_marker overlaps grad_out or grad_mask");
    return run_bwd(dtype, codes, grad_out, grad_marker, grad_mask, shape, n_images, image_stride, n_steps,
                   (hipStream_t)hip_stream);
}

// Source ids are element offsets within an image, below 2^31.
static int validate_sources_shape(const gc_shape &s) {
    if (s.width > 0 && s.height > 0 && (s.height - 1) * s.pitch + s.width > (int64_t)INT32_MAX)
        return fail(GC_ERR_UNSUPPORTED, "source ids need images of at most 2^31 - 1 elements per image");
    return GC_OK;
}

int gc_geodesic_chain_fwd_sources(gc_dtype dtype, gc_op op, const void *marker, const void *mask, void *out,
                                  uint32_t *sources, gc_shape shape, int32_t n_images, int64_t image_stride,
                                  int64_t n_steps, void *hip_stream) {
    GC_CHECK_DTYPE(dtype);
    GC_CHECK_OP(op);
    g_last_error.clear();
    int rc = validate_batch(dtype, shape, n_images, image_stride, n_steps);
    if (rc != GC_OK) return rc;
    rc = validate_sources_shape(shape);
    if (rc != GC_OK) return rc;
    const bool empty = shape.width == 0 || shape.height == 0 || n_images == 0;
    if (empty) return GC_OK;
    if (!marker || !mask || !out || !sources) return fail(GC_ERR_INVALID_ARG, "null pointer");
    const size_t es = elem_size(dtype);
    const auto eo = batch_extent(out, shape, n_images, image_stride, es);
    const auto es_ = batch_extent(sources, shape, n_images, image_stride, 4);
    if (overlap(eo, batch_extent(mask, shape, n_images, image_stride, es)))
        return fail(GC_ERR_ALIAS, "out overlaps mask");
    if (out != marker && overlap(eo, batch_extent(marker, shape, n_images, image_stride, es)))
        return fail(GC_ERR_ALIAS, "out partially overlaps marker");
    if (overlap(es_, eo) || overlap(es_, batch_extent(marker, shape, n_images, image_stride, es)) ||
        overlap(es_, batch_extent(mask, shape, n_images, image_stride, es)))
        return fail(GC_ERR_ALIAS, "sources overlaps an image");
    return run_fwd_sources(dtype, enum_bits(&op), marker, mask, out, sources, shape, n_images, image_stride,
                           n_steps, (hipStream_t)hip_stream);
}

int gc_geodesic_chain_bwd_sources(gc_dtype dtype, const uint32_t *sources, const void *grad_out,
                                  void *grad_marker, void *grad_mask, gc_shape shape, int32_t n_images,
                                  int64_t image_stride, void *hip_stream) {
    GC_CHECK_DTYPE(dtype);
    g_last_error.clear();
    int rc = validate_batch(dtype, shape, n_images, image_stride, 0);
    if (rc != GC_OK) return rc;
    rc = validate_sources_shape(shape);
    if (rc != GC_OK) return rc;
    const bool empty = shape.width == 0 || shape.height == 0 || n_images == 0;
    if (empty) return GC_OK;
    if (!sources || !grad_out || !grad_marker || !grad_mask) return fail(GC_ERR_INVALID_ARG, "null pointer");
    const size_t es = elem_size(dtype);
    const auto egm = batch_extent(grad_marker, shape, n_images, image_stride, es);
    const auto egk = batch_extent(grad_mask, shape, n_images, image_stride, es);
    const auto ego = batch_extent(grad_out, shape, n_images, image_stride, es);
    if (overlap(egm, ego) || overlap(egm, egk) || overlap(egk, ego))
        return fail(GC_ERR_ALIAS, "grad_marker, grad_mask and grad_out must not overlap");
    const auto es_ = batch_extent(sources, shape, n_images, image_stride, 4);
    if (overlap(es_, egm) || overlap(es_, egk) || overlap(es_, ego))
        return fail(GC_ERR_ALIAS, "sources overlaps a gradient");
    return run_bwd_sources(dtype, sources, grad_out, grad_marker, grad_mask, shape, n_images, image_stride,
                           (hipStream_t)hip_stream);
}

int gc_plan_create(gc_dtype dtype, gc_op op, const gc_item *items, int32_t n_items, gc_plan **plan_out) {
    GC_CHECK_DTYPE(dtype);
    GC_CHECK_OP(op);
    g_last_error.clear();
    return plan_build(dtype, (int)op, items, n_items, plan_out, nullptr);
}

int gc_plan_tune(gc_plan *plan, double *best_ms) {
    g_last_error.clear();
    if (!plan) return fail(GC_ERR_INVALID_ARG, "plan is NULL");
    int dev = 0;
    GC_HIP(hipGetDevice(&dev));
    if (dev != plan->device) return fail(GC_ERR_INVALID_ARG, "plan belongs to device %d", plan->device);
    if (!plan->stab_imgs.empty())
        return fail(GC_ERR_UNSUPPORTED, "plans with run-to-stability items keep the built-in launch shape");
    if (plan->launched) GC_HIP(hipStreamSynchronize(plan->last_stream));
    const size_t es = elem_size(plan->dtype);
    const size_t n = plan->items.size();
    // Scratch images of the same shapes and chain lengths: the kernels'
    // cost does not depend on the pixel values, and the caller's buffers
    // (in-place items included) are never touched.
    std::vector<size_t> off(n);
    size_t total = 0;
    for (size_t i = 0; i < n; ++i) {
        const gc_shape &sh = plan->items[i].shape;
        off[i] = total;
        total += 3 * (((size_t)(sh.width * sh.height) * es + 255) & ~(size_t)255);
    }
    void *buf = nullptr;
    if (total && hipMalloc(&buf, total) != hipSuccess) {
        (void)hipGetLastError();
        return fail(GC_ERR_NO_MEMORY, "tuning scratch of %zu bytes", total);
    }
    if (total) GC_HIP(hipMemset(buf, 0, total));
    std::vector<gc_item> scratch(n);
    for (size_t i = 0; i < n; ++i) {
        const gc_item &it = plan->items[i];
        const size_t plane = ((size_t)(it.shape.width * it.shape.height) * es + 255) & ~(size_t)255;
        char *b = static_cast<char *>(buf) + off[i];
        scratch[i].marker = b;
        scratch[i].mask = it.mask ? b + plane : nullptr;
        scratch[i].out = b + 2 * plane;
        scratch[i].shape = gc_shape{it.shape.width, it.shape.height, it.shape.width};
        scratch[i].n_steps = it.n_steps;
    }
    PlanChoice best;
    double best_t = 1e300;
    const int fams[] = {FAM_128W, FAM_128, FAM_96W, FAM_96};
    for (int fam : fams) {
        for (int k = 12; k <= std::min(28, persistent_kmax(fam)); k += 4) {
            PlanChoice ch;
            ch.fam = fam;
            for (size_t i = 0; i < n; ++i) {
                const int64_t ni = plan->items[i].n_steps;
                ch.k.push_back(ni > 0 && ni < k ? (int)ni : k);
            }
            gc_plan *cand = nullptr;
            if (plan_build(plan->dtype, plan->op, scratch.data(), (int32_t)n, &cand, &ch) != GC_OK) continue;
            double ms = 0;
            const int rc = plan_time(cand, 2, &ms);
            plan_free(cand);
            if (rc != GC_OK) {
                if (buf) (void)hipFree(buf);
                return rc;
            }
            if (ms < best_t) {
                best_t = ms;
                best = ch;
            }
        }
    }
    if (buf) (void)hipFree(buf);
    if (best_t == 1e300) return fail(GC_ERR_UNSUPPORTED, "no launch shape could be built for this batch");
    gc_plan *tuned = nullptr;
    int rc = plan_build(plan->dtype, plan->op, plan->items.data(), (int32_t)n, &tuned, &best);
    if (rc != GC_OK) return rc;
    std::swap(*plan, *tuned);   // the caller's handle now holds the tuned plan
    plan_free(tuned);
    if (best_ms) *best_ms = best_t;
    return GC_OK;
}

int gc_plan_launch(gc_plan *plan, void *hip_stream) {
    g_last_error.clear();
    if (!plan) return fail(GC_ERR_INVALID_ARG, "plan is NULL");
    int dev = 0;
    GC_HIP(hipGetDevice(&dev));
    if (dev != plan->device) return fail(GC_ERR_INVALID_ARG, "plan belongs to device %d", plan->device);
    hipStream_t st = (hipStream_t)hip_stream;
    for (size_t i = 0; i < plan->items.size(); ++i) {
        const gc_item &it = plan->items[i];
        const bool empty = it.shape.width == 0 || it.shape.height == 0;
        plan->steps[i] = it.n_steps >= 0 ? it.n_steps : (empty ? 0 : -1);
    }
    if (plan->stab_imgs.empty()) {
        const int pr = prof_begin(st, 0);
        GC_HIP(hipGraphLaunch(plan->exec, st));
        prof_end(pr, st);
        plan->last_stream = st;
        plan->launched = true;
        return GC_OK;
    }
    // Run-to-stability items: each replay runs STAB_BLOCKS blocks of STAB_K
    // steps of every active image and records, per block, the OR over its
    // tiles of the per-step change bits.  Once a full step changes nothing the
    // state is a fixed point, so the bits of an image form a run of ones: the
    // first zero is its step count, and the state after the replay is the
    // result.  Images that changed at every step continue from their output
    // in the next replay; converged and fixed-length images sit it out.
    plan->last_stream = st;
    plan->launched = true;
    std::vector<geochain::PlanImage> tab = plan->imgs_init;
    const size_t tab_bytes = tab.size() * sizeof(geochain::PlanImage);
    GC_HIP(hipMemcpyAsync(plan->images_d, tab.data(), tab_bytes, hipMemcpyHostToDevice, st));
    const size_t n_stab = plan->stab_imgs.size();
    std::vector<int64_t> changed(n_stab, 0);
    std::vector<char> done(n_stab, 0);
    size_t left = n_stab;
    while (left > 0) {
        GC_HIP(hipGraphLaunch(plan->exec, st));
        GC_HIP(hipStreamSynchronize(st));
        if (*plan->error_h) return fail(GC_ERR_HIP, "a dependency wait inside the batch kernel hit its bound");
        for (auto &im : tab) im.active = 0;  // fixed-length images are complete after the first replay
        for (size_t q = 0; q < n_stab; ++q) {
            if (done[q]) continue;
            const int j = plan->stab_imgs[q];
            const uint32_t *w = plan->change_h + q * STAB_BLOCKS;
            const uint32_t full = (uint32_t)((1ull << tab[j].k) - 1);
            bool stable = false;
            for (int b = 0; b < STAB_BLOCKS && !stable; ++b) {
                if (w[b] == full) {
                    changed[q] += tab[j].k;
                } else {
                    changed[q] += __builtin_ctz(~w[b]);
                    stable = true;
                }
            }
            const gc_item &it = plan->items[plan->img_item[j]];
            if (stable) {
                done[q] = 1;
                --left;
                plan->steps[plan->img_item[j]] = changed[q];
            } else if (changed[q] > it.shape.width * it.shape.height + 1) {
                // a reconstruction changes something at each step along a path
                // of distinct pixels, so this bound is never reached
                return fail(GC_ERR_NOT_CONVERGED, "item %d did not converge in %lld steps", plan->img_item[j],
                            (long long)changed[q]);
            } else {
                tab[j].active = 1;
                tab[j].marker = tab[j].out;  // continue from this replay's result
            }
        }
        if (left > 0) GC_HIP(hipMemcpyAsync(plan->images_d, tab.data(), tab_bytes, hipMemcpyHostToDevice, st));
    }
    return GC_OK;
}

int gc_plan_steps(const gc_plan *plan, int64_t *steps) {
    g_last_error.clear();
    if (!plan || !steps) return fail(GC_ERR_INVALID_ARG, "plan or steps is NULL");
    for (size_t i = 0; i < plan->steps.size(); ++i) steps[i] = plan->steps[i];
    return GC_OK;
}

int gc_plan_status(gc_plan *plan) {
    g_last_error.clear();
    if (!plan) return fail(GC_ERR_INVALID_ARG, "plan is NULL");
    if (!plan->launched) return GC_OK;
    GC_HIP(hipStreamSynchronize(plan->last_stream));
    if (*plan->error_h) return fail(GC_ERR_HIP, "a dependency wait inside the batch kernel hit its bound");
    return GC_OK;
}

int gc_plan_info(const gc_plan *plan, int64_t *px_steps, int64_t *work_items, int32_t *workgroups,
                 int32_t *tile, int32_t *block_steps) {
    g_last_error.clear();
    if (!plan) return fail(GC_ERR_INVALID_ARG, "plan is NULL");
    if (px_steps) *px_steps = plan->px_steps;
    if (work_items) *work_items = plan->n_items;
    if (workgroups) *workgroups = plan->grid;
    if (tile) *tile = plan->fam;
    if (block_steps) *block_steps = plan->max_k;
    return GC_OK;
}

int gc_plan_destroy(gc_plan *plan) {
    g_last_error.clear();
    if (!plan) return GC_OK;
    if (plan->launched) (void)hipStreamSynchronize(plan->last_stream);
    plan_free(plan);
    return GC_OK;
}

int gc_autotune(gc_dtype dtype, gc_op op, int32_t geodesic, int64_t width, int64_t height, int32_t *best_tile,
                int32_t *best_k) {
    GC_CHECK_DTYPE(dtype);
    GC_CHECK_OP(op);
    g_last_error.clear();
    if (elem_size(dtype) == 0) return fail(GC_ERR_INVALID_ARG, "unknown dtype");
    if (op != GC_DILATE && op != GC_ERODE) return fail(GC_ERR_INVALID_ARG, "unknown op");
    if (width < 1 || height < 1 || width > 16384 || height > 16384)
        return fail(GC_ERR_INVALID_ARG, "tuning sizes are 1..16384");
    // Tune on the size class's upper corner.
    const TuneKey key = tune_key(dtype, (int)op, geodesic, width, height);
    TuneVal tv;
    int rc = autotune(dtype, (int)op, geodesic, int64_t(1) << key.cw, int64_t(1) << key.ch, &tv);
    if (rc != GC_OK) return rc;
    {
        std::lock_guard<std::mutex> g(g_autotune_mu);
        g_autotune[key] = tv;
    }
    if (best_tile) *best_tile = tv.best_fam;
    if (best_k) *best_k = tv.k[tv.best_fam];
    return GC_OK;
}

int gc_autotune_clear(void) {
    std::lock_guard<std::mutex> g(g_autotune_mu);
    g_autotune.clear();
    return GC_OK;
}

static_assert(GC_TUNE_FAMILIES == NUM_FAMS, "one tuning record slot per tile family");

int gc_autotune_export(gc_tune_entry *out, int32_t cap, int32_t *count) {
    g_last_error.clear();
    if (!count) return fail(GC_ERR_INVALID_ARG, "count is NULL");
    if (cap < 0) return fail(GC_ERR_INVALID_ARG, "cap < 0");
    if (cap > 0 && !out) return fail(GC_ERR_INVALID_ARG, "out is NULL");
    std::lock_guard<std::mutex> g(g_autotune_mu);
    int32_t i = 0;
    for (const auto &kv : g_autotune) {
        if (i >= cap) break;
        gc_tune_entry e{};
        e.dtype = kv.first.dtype;
        e.op = kv.first.op;
        e.geodesic = kv.first.geodesic;
        e.log2_width = kv.first.cw;
        e.log2_height = kv.first.ch;
        e.best_tile = kv.second.best_fam;
        for (int f = 0; f < NUM_FAMS; ++f) {
            e.k[f] = kv.second.k[f];
            e.rate[f] = kv.second.rate[f];
        }
        out[i++] = e;
    }
    *count = (int32_t)g_autotune.size();
    return GC_OK;
}

int gc_autotune_import(const gc_tune_entry *entries, int32_t n) {
    g_last_error.clear();
    if (n < 0) return fail(GC_ERR_INVALID_ARG, "n < 0");
    if (n > 0 && !entries) return fail(GC_ERR_INVALID_ARG, "entries is NULL");
    for (int32_t i = 0; i < n; ++i) {
        const gc_tune_entry &e = entries[i];
        if (e.dtype != GC_U8 && e.dtype != GC_F32 && e.dtype != GC_F64)
            return fail(GC_ERR_INVALID_ARG, "record %d: unknown dtype %d", i, e.dtype);
        if (e.op != GC_DILATE && e.op != GC_ERODE) return fail(GC_ERR_INVALID_ARG, "record %d: unknown op %d", i, e.op);
        if (e.geodesic != 0 && e.geodesic != 1)
            return fail(GC_ERR_INVALID_ARG, "record %d: geodesic must be 0 or 1", i);
        if (e.log2_width < 0 || e.log2_width > 14 || e.log2_height < 0 || e.log2_height > 14)
            return fail(GC_ERR_INVALID_ARG, "record %d: size class outside 2^0..2^14", i);
        if (e.best_tile < 0 || e.best_tile >= NUM_FAMS)
            return fail(GC_ERR_INVALID_ARG, "record %d: unknown tile family %d", i, e.best_tile);
        for (int f = 0; f < NUM_FAMS; ++f) {
            if (e.k[f] < 0 || e.k[f] > 63) return fail(GC_ERR_INVALID_ARG, "record %d: steps per block outside 0..63", i);
            if (!(e.rate[f] >= 0.0) || !std::isfinite(e.rate[f]))
                return fail(GC_ERR_INVALID_ARG, "record %d: rates must be finite and >= 0", i);
        }
        if (e.k[e.best_tile] < 1) return fail(GC_ERR_INVALID_ARG, "record %d: the chosen family has no steps per block", i);
    }
    std::lock_guard<std::mutex> g(g_autotune_mu);
    for (int32_t i = 0; i < n; ++i) {
        const gc_tune_entry &e = entries[i];
        TuneVal tv;
        tv.best_fam = e.best_tile;
        for (int f = 0; f < NUM_FAMS; ++f) {
            tv.k[f] = e.k[f];
            tv.rate[f] = e.rate[f];
        }
        g_autotune[TuneKey{e.dtype, e.op, e.geodesic, e.log2_width, e.log2_height}] = tv;
    }
    return GC_OK;
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

int gc_validate_values(gc_dtype dtype, const void *image, gc_shape shape, int32_t allow_inf, void *hip_stream) {
    GC_CHECK_DTYPE(dtype);
    g_last_error.clear();
    int rc = validate_shape(dtype, shape);
    if (rc != GC_OK) return rc;
    if (dtype == GC_U8 || shape.width == 0 || shape.height == 0) return GC_OK;
    if (!image) return fail(GC_ERR_INVALID_ARG, "null image pointer");
    uint32_t found = 0;
    rc = dtype == GC_F32 ? run_value_scan_t<float>((const float *)image, shape, &found, hip_stream)
                         : run_value_scan_t<double>((const double *)image, shape, &found, hip_stream);
    if (rc != GC_OK) return rc;
    if (found & 1u) return fail(GC_ERR_INVALID_ARG, "the image holds a NaN");
    if ((found & 2u) && !allow_inf) return fail(GC_ERR_INVALID_ARG, "the image holds an infinity");
    return GC_OK;
}

int gc_set_window_path(int32_t min_steps) {
    if (min_steps < -1) return fail(GC_ERR_INVALID_ARG, "min_steps < -1");
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_window_min_steps = min_steps;
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
