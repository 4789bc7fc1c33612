// chain_launch.hpp -- launch shapes of the chain kernel (chain_block.hpp):
// the tile families (region layout per workgroup), the choice of family and
// steps per launch for an image and chain length, the tile geometry, and
// the launch wrappers.  Host code, included once by geochain.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>

#include "chain_block.hpp"

namespace geochain {

// ---------------------------------------------------------------------------
// tuning
// ---------------------------------------------------------------------------
static std::mutex g_tune_mu;
static int g_tune_k = 0;      // 0 = built-in
static int g_tune_tile = -1;  // -1 = built-in

enum { FAM_128 = 0, FAM_64 = 1, FAM_128W = 2, FAM_96 = 3, FAM_96W = 4, NUM_FAMS = 5 };

template <typename T, int FAM> struct Family;
// G: column groups per wave (1: 64 lanes across; 2: two 32-lane groups
// stacked vertically, see chain_block_body_g2).
// 128 x 128 region: 2 columns per lane; 8 waves of 16 rows (16 waves of 8
// rows for f64, whose registers are twice as wide).
template <typename T> struct Family<T, FAM_128> {
    static constexpr int CW = 2;
    static constexpr int RPW = sizeof(T) == 8 ? 8 : 16;
    static constexpr int NW = sizeof(T) == 8 ? 16 : 8;
    static constexpr int G = 1;
};
// 64 x 64 region for small images: 1 column per lane, 8 waves of 8 rows.
template <typename T> struct Family<T, FAM_64> {
    static constexpr int CW = 1;
    static constexpr int RPW = 8;
    static constexpr int NW = 8;
    static constexpr int G = 1;
};

// 128 x 128 region with twice the waves: 16 waves of 8 rows (f64: 16 waves
// of 8 rows as well, i.e. the same as FAM_128).
template <typename T> struct Family<T, FAM_128W> {
    static constexpr int CW = 2;
    static constexpr int RPW = 8;
    static constexpr int NW = 16;
    static constexpr int G = 1;
};
// 96 x 96 region, two 32-lane groups of 3 columns: 8 waves of 2 x 6 rows.
template <typename T> struct Family<T, FAM_96> {
    static constexpr int CW = 3;
    static constexpr int RPW = 6;
    static constexpr int NW = 8;
    static constexpr int G = 2;
};
// 96 x 96 region with 16 waves of 2 x 3 rows.
template <typename T> struct Family<T, FAM_96W> {
    static constexpr int CW = 3;
    static constexpr int RPW = 3;
    static constexpr int NW = 16;
    static constexpr int G = 2;
};

static int region_side(int fam) {
    switch (fam) {
        case FAM_64: return 64;
        case FAM_96:
        case FAM_96W: return 96;
        default: return 128;
    }
}

struct Plan1 {
    int fam;
    int k;
};

// Built-in choice of tile family and steps per launch.
static Plan1 choose_plan(const gc_shape &s, int64_t n, bool detect) {
    Plan1 p;
    const int64_t side = std::max(s.width, s.height);
    p.fam = side >= 384 ? FAM_128W : FAM_64;
    p.k = region_side(p.fam) == 128 ? 32 : 16;
    // Short chains of known length on large images: one launch of 128 x 128
    // regions has few, large cores (81 workgroups for one step at 1024^2);
    // smaller regions spread the same work over more CUs.  Measured at
    // 1024^2 u8: 64 x 64 regions are fastest up to 10 steps, 96 x 96 up to 16.
    if (side >= 384 && n > 0 && n <= 16) {
        p.fam = n <= 10 ? FAM_64 : FAM_96W;
        p.k = (int)n;
    }
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
// dispatch
// ---------------------------------------------------------------------------
using LaunchFn = void (*)(const BlockArgs &, int grid, hipStream_t);

// One workgroup per tile.  A grid holds fewer than 2^32 work-items, so the
// tiles of a large image go out in launches of at most MAX_TILES_PER_LAUNCH
// (2^30 work-items), each told its first tile.  The tiles of one block of
// steps are independent (they read src and write disjoint cores of dst), so
// consecutive launches on the stream compute exactly what one would.
constexpr int MAX_TILES_PER_LAUNCH = 1 << 20;

template <typename T, int OP, int MODE, bool DETECT, int FAM>
static void launch_block(const BlockArgs &a, int grid, hipStream_t st) {
    using F = Family<T, FAM>;
    for (int t0 = 0; t0 < grid; t0 += MAX_TILES_PER_LAUNCH) {
        BlockArgs b = a;
        b.tile0 = t0;
        hipLaunchKernelGGL((chain_block_kernel<T, OP, MODE, DETECT, F::CW, F::RPW, F::NW, F::G>),
                           dim3(std::min(grid - t0, MAX_TILES_PER_LAUNCH)), dim3(64 * F::NW), 0, st, b);
    }
}

template <typename T, int OP, int MODE, bool DETECT>
static LaunchFn pick_fam(int fam) {
    switch (fam) {
        case FAM_64: return &launch_block<T, OP, MODE, DETECT, FAM_64>;
        case FAM_128W: return &launch_block<T, OP, MODE, DETECT, FAM_128W>;
        case FAM_96: return &launch_block<T, OP, MODE, DETECT, FAM_96>;
        case FAM_96W: return &launch_block<T, OP, MODE, DETECT, FAM_96W>;
        default: return &launch_block<T, OP, MODE, DETECT, FAM_128>;
    }
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

// Mixed chains (a dilation or an erosion per step): 128 x 128 regions, u8
// and f32 (the f64 body would spill registers with four step copies).
static LaunchFn pick_mixed(gc_dtype d) {
    switch (d) {
        case GC_U8: return &launch_block<uint8_t, OP_DILATE, MODE_MIXED, false, FAM_128W>;
        case GC_F32: return &launch_block<float, OP_DILATE, MODE_MIXED, false, FAM_128W>;
        default: return nullptr;
    }
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

}  // namespace geochain
