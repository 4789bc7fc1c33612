// grad_block.hpp -- kernels for differentiating a geodesic chain (not part
// of the paper, which has no backward pass).
//
// Every output of a geodesic step is a copy of exactly one input value: the
// extremal pixel of the clipped 3x3 window (Eq. 1-2) or the mask (Eq. 3).
// The forward kernel records, per step and pixel, a code naming that source:
//   code (dy+1)*3 + (dx+1)  the FIRST extremal neighbour in raster (dy, dx)
//                           order (ties between neighbours go to the earlier
//                           one, as max_pool2d's indices do);
//   code 9                  the mask won the clamp (ties go to the mask).
// The first extremum in raster order is what a row pass followed by a column
// pass yields when each keeps its earliest extremum on ties (the 3x3 square
// decomposes as in Section 3.1).  The backward kernel is a GATHER: pixel q
// collects the upstream gradient of every neighbour p whose code points at
// q, visiting p in raster order (the order a raster-order scatter delivers
// them), and the mask gradient collects g(q) where code(q) == 9.
//
// Both kernels are temporal-blocked: up to GB_K steps per launch on a region
// of 64 columns (one per lane) and NW * 8 rows with a GB_K-pixel halo.  Each
// wave keeps its 8 rows in registers; the left and right columns come from
// the adjacent lanes by DPP and only the wave's two edge rows go through
// LDS, one barrier per step.  A wave whose rows are all further than the
// remaining steps from the core only takes the barriers.
//
//   block_codes_kernel  k steps forward; the codes of the core pixels are
//                       staged in LDS and stored as 16-byte rows;
//   block_bwd_kernel    k steps backward with the k code planes in LDS; the
//                       mask gradient is accumulated in registers starting
//                       from the stored value, so its additions happen in the
//                       same order (steps from last to first) as in a
//                       one-step-at-a-time reverse pass.
//
// Values must be finite: a pixel outside the image is represented by the
// neutral extremum (-inf for dilation), which must never tie with a real
// value.  Codes are stored densely: codes[image][step][y][width] bytes.
// Pixels on the region's outer edge (lanes 0 and 63, the first and last
// wave's outer rows) see wrong neighbours; an error moves one pixel per step
// and the core starts GB_K pixels in, so the core is exact.  One launch
// covers a batch of images (grid.z = image).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "chain_block.hpp"

namespace geochain {

constexpr uint8_t CODE_MASK = 9;
constexpr uint8_t CODE_NONE = 255;

// Block of a workgroup: the grid (column tile, row tile, image) is relabelled
// XCD by XCD (xcd_tile), so neighbouring tiles, whose regions overlap, run
// on one XCD and share its L2.
struct GradBlock {
    int bx, by, img;
};
__device__ __forceinline__ GradBlock grad_block() {
    const unsigned gx = gridDim.x, gy = gridDim.y;
    const unsigned lin = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    const unsigned t = (unsigned)xcd_tile(lin, gx * gy * gridDim.z);
    return GradBlock{(int)(t % gx), (int)((t / gx) % gy), (int)(t / (gx * gy))};
}

template <int OP, typename T>
__device__ __forceinline__ bool better(T a, T b) {
    return OP == OP_DILATE ? (a > b) : (a < b);
}

// Extremum of two values (max for dilation, min for erosion); values are
// finite, so max3/min3 forms apply.
template <int OP, typename T>
__device__ __forceinline__ T extremum(T a, T b) {
    if constexpr (OP == OP_DILATE) return a > b ? a : b;
    else return a < b ? a : b;
}

// Value of the adjacent lane (lane = region column): WAVE_SHR1 gives column
// x - 1, WAVE_SHL1 column x + 1.  Lanes 0 / 63 receive 0: they are the
// region's outer columns, whose results are wrong anyway and never reach the
// core (an error moves one column per step, the core starts GB_K columns in).
// Zero fill lets the compiler fold the shift into the consuming compare/add.
template <int CTRL>
__device__ __forceinline__ int gb_shift(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true);
}
template <int CTRL>
__device__ __forceinline__ float gb_shift(float v) {
    return __builtin_bit_cast(float, gb_shift<CTRL>(__builtin_bit_cast(int, v)));
}
template <int CTRL>
__device__ __forceinline__ double gb_shift(double v) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)gb_shift<CTRL>((int)(uint32_t)u);
    const uint32_t hi = (uint32_t)gb_shift<CTRL>((int)(uint32_t)(u >> 32));
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Region: GB_RW = 64 columns, one per lane; wave w holds rows [8w, 8w + 8).
// Core: (64 - 2 GB_K) columns by (rows - 2 GB_K) rows.  Every wave walks the
// same rows in the same order, so band tests are uniform per wave.
constexpr int GB_K = 8;                        // largest steps per launch
constexpr int GB_RW = 64;                      // region width (lanes)
constexpr int GB_CX = GB_RW - 2 * GB_K;        // core width (48)
constexpr int GB_WR = 8;                       // rows per wave

template <typename T> struct GradTile {
    // f64 tiles are shorter so that the backward's code planes and 64-bit
    // edge exchange still let two workgroups share a CU's LDS.
    static constexpr int NW = sizeof(T) == 8 ? 12 : 16;   // waves
    static constexpr int RH = NW * GB_WR;                 // region height
    static constexpr int CY = RH - 2 * GB_K;              // core height
    static constexpr int THREADS = 64 * NW;
    // Waves per SIMD the codes kernel is compiled for: two f32 workgroups
    // per CU (at most 64 VGPRs); f64 keeps its register budget.
    static constexpr int CODES_WAVES_PER_SIMD = sizeof(T) == 8 ? 1 : 8;
};

struct GradBlockArgs {
    const void *src;          // state (codes kernel) or upstream gradient (bwd) at the block's start
    const void *mask;         // mask (codes kernel)
    void *dst;                // state / gradient at the block's end
    void *g_mask;             // bwd: mask gradient, accumulated
    uint8_t *codes;           // codes of the block's first step, image 0
    int64_t codes_step;       // bytes between steps (height * width)
    int64_t codes_image;      // bytes between images (n_steps * height * width)
    int64_t image_stride;     // elements between images of src / mask / dst / g_mask
    int64_t pitch;
    int32_t width, height;
    int32_t k;                // steps in this launch (<= GB_K)
};

// Stores one step's core codes (GB_CX x CY bytes staged in LDS) as 16-byte
// pieces: 3 threads per row.
template <int CY>
__device__ __forceinline__ void gb_store_codes(const uint8_t (*sc)[GB_CX], uint8_t *codes, int x0, int y0,
                                               int width, int height) {
    const int row = threadIdx.x / 3, seg = (threadIdx.x % 3) * 16;
    if (row >= CY) return;
    const int y = y0 + row, x = x0 + seg;
    if (y >= height || x >= width) return;
    uint8_t *p = codes + (int64_t)y * width + x;
    if (x + 16 <= width && ((uintptr_t)p & 15) == 0) {
        *reinterpret_cast<uint4 *>(p) = *reinterpret_cast<const uint4 *>(&sc[row][seg]);
    } else {
        for (int i = 0; i < 16 && x + i < width; ++i) p[i] = sc[row][seg + i];
    }
}

// Rows a wave must still compute at step s of a k-step launch: those whose
// result is needed (within k-1-s of the core) and, one further out, those
// whose row-pass result or gradient a needed edge row reads from this wave.
// A wave holding any of them computes all of its rows; the others only take
// the barriers: what they leave stale lies at least k-s rows from the core
// and moves at most one row per remaining step, so it never reaches it.
template <int CY>
__device__ __forceinline__ bool gb_wave_busy(int w, int k, int s) {
    const int lo = GB_K - (k - s), hi = GB_K + CY + (k - s);
    return w * GB_WR + GB_WR > lo && w * GB_WR < hi;
}

// Forward: k steps of the chain recording every core pixel's source code.
// Each wave keeps its GB_WR rows of the state in registers (lane = column);
// the row pass takes the neighbour columns by DPP, the column pass reads the
// rows above and below from the wave's own registers, and only the two edge
// rows' row-pass results (value and index) go through LDS, one barrier per
// step.  The codes of a step are staged in LDS (double-buffered) and stored
// as 16-byte rows after the next step's barrier.
template <typename T, int OP>
__global__ __launch_bounds__(GradTile<T>::THREADS, GradTile<T>::CODES_WAVES_PER_SIMD) void block_codes_kernel(
    GradBlockArgs a) {
    using B = Bounds<T, OP>;
    using G = GradTile<T>;
    constexpr int CY = G::CY, NW = G::NW;
    __shared__ T xv[2][NW][2][GB_RW];        // edge rows' row-pass values
    __shared__ uint8_t xi[2][NW][2][GB_RW];  // and their dx indices
    __shared__ __attribute__((aligned(16))) uint8_t sc[2][CY][GB_CX];
    const GradBlock blk = grad_block();
    const int img = blk.img;
    const T *src = static_cast<const T *>(a.src) + img * a.image_stride;
    const T *msk = static_cast<const T *>(a.mask) + img * a.image_stride;
    T *dst = static_cast<T *>(a.dst) + img * a.image_stride;
    uint8_t *codes = a.codes + img * a.codes_image;
    const int x0 = blk.bx * GB_CX, y0 = blk.by * CY;  // core origin
    const int rx0 = x0 - GB_K, ry0 = y0 - GB_K;               // region origin
    const int x = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wa = w > 0 ? w - 1 : NW - 1, wb = w < NW - 1 ? w + 1 : 0;  // region edge: harmless wrap
    const int gx = rx0 + x;
    const bool xin = (unsigned)gx < (unsigned)a.width;
    const bool col_core = (unsigned)(x - GB_K) < (unsigned)GB_CX;

    T v[GB_WR], m[GB_WR];
#pragma unroll
    for (int r = 0; r < GB_WR; ++r) {
        const int y = ry0 + w * GB_WR + r;
        const bool in = xin && (unsigned)y < (unsigned)a.height;
        const int64_t off = (int64_t)y * a.pitch + gx;
        v[r] = in ? src[off] : B::bottom();
        m[r] = in ? msk[off] : B::bottom();
    }

    const int k = a.k;
    for (int s = 0; s < k; ++s) {
        const int par = s & 1;
        const bool busy = gb_wave_busy<CY>(w, k, s);
        T h[GB_WR];
        int ix[GB_WR];
        if (busy) {
            // row pass: first extremum of (x-1, x, x+1) and its dx index
#pragma unroll
            for (int r = 0; r < GB_WR; ++r) {
                // the first of (x-1, x, x+1) equal to their extremum is the
                // first extremum in raster order
                const T c = v[r];
                const T left = gb_shift<DPP_WAVE_SHR1>(c);
                const T right = gb_shift<DPP_WAVE_SHL1>(c);
                const T best = extremum<OP>(extremum<OP>(left, c), right);
                h[r] = best;
                // two unconditional selects (a nested conditional of this
                // shape compiles to divergent branches)
                const int t = c == best ? 1 : 2;
                ix[r] = left == best ? 0 : t;
            }
            xv[par][w][0][x] = h[0];
            xi[par][w][0][x] = (uint8_t)ix[0];
            xv[par][w][1][x] = h[GB_WR - 1];
            xi[par][w][1][x] = (uint8_t)ix[GB_WR - 1];
        }
        __syncthreads();
        // the previous step's codes are complete: store them
        if (s > 0) gb_store_codes<CY>(sc[par ^ 1], codes + (s - 1) * a.codes_step, x0, y0, a.width, a.height);
        if (busy) {
            const T ha = xv[par][wa][1][x], hb = xv[par][wb][0][x];
            const int ia = xi[par][wa][1][x], ib = xi[par][wb][0][x];
            // column pass: first extremum of rows y-1, y, y+1 in raster order,
            // then the clamp (the mask wins ties)
#pragma unroll
            for (int r = 0; r < GB_WR; ++r) {
                const T hu = r == 0 ? ha : h[r - 1];
                const int iu = r == 0 ? ia : ix[r - 1];
                const T hd = r == GB_WR - 1 ? hb : h[r + 1];
                const int id = r == GB_WR - 1 ? ib : ix[r + 1];
                const T best = extremum<OP>(extremum<OP>(hu, h[r]), hd);
                const int t = h[r] == best ? 3 + ix[r] : 6 + id;
                const int code = hu == best ? iu : t;
                const bool mask_wins = OP == OP_DILATE ? !(best < m[r]) : !(best > m[r]);
                v[r] = mask_wins ? m[r] : best;
                const int cy = w * GB_WR + r - GB_K;
                if ((unsigned)cy < (unsigned)CY && col_core)
                    sc[par][cy][x - GB_K] = mask_wins ? CODE_MASK : (uint8_t)code;
            }
        }
    }
    __syncthreads();
    gb_store_codes<CY>(sc[(k - 1) & 1], codes + (k - 1) * a.codes_step, x0, y0, a.width, a.height);
    // core of the final state
    if (col_core && xin) {
#pragma unroll
        for (int r = 0; r < GB_WR; ++r) {
            const int ly = w * GB_WR + r, y = ry0 + ly;
            if ((unsigned)(ly - GB_K) < (unsigned)CY && y < a.height) dst[(int64_t)y * a.pitch + gx] = v[r];
        }
    }
}

// Backward: k steps of the reverse gather.  Each wave keeps its rows'
// gradients in registers; the codes of the k steps sit in LDS; the two edge
// rows' gradients go through LDS each step.  Pixel q takes, in raster
// order, the upstream gradient of each neighbour p = q + d whose code names
// -d, and adds its own gradient to the mask gradient where its code is
// CODE_MASK.
template <typename T>
__global__ __launch_bounds__(GradTile<T>::THREADS) void block_bwd_kernel(GradBlockArgs a) {
    using G = GradTile<T>;
    constexpr int RH = G::RH, CY = G::CY, NW = G::NW;
    __shared__ __attribute__((aligned(16))) uint8_t scd[GB_K][RH][GB_RW];
    __shared__ T xg[2][NW][2][GB_RW];
    const GradBlock blk = grad_block();
    const int img = blk.img;
    const T *gin = static_cast<const T *>(a.src) + img * a.image_stride;
    T *gout = static_cast<T *>(a.dst) + img * a.image_stride;
    T *gm = static_cast<T *>(a.g_mask) + img * a.image_stride;
    const uint8_t *codes = a.codes + img * a.codes_image;
    const int x0 = blk.bx * GB_CX, y0 = blk.by * CY;
    const int rx0 = x0 - GB_K, ry0 = y0 - GB_K;
    const int x = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wa = w > 0 ? w - 1 : NW - 1, wb = w < NW - 1 ? w + 1 : 0;
    const int gx = rx0 + x;
    const bool xin = (unsigned)gx < (unsigned)a.width;
    const int k = a.k;

    T g[GB_WR];
#pragma unroll
    for (int r = 0; r < GB_WR; ++r) {
        const int y = ry0 + w * GB_WR + r;
        const bool in = xin && (unsigned)y < (unsigned)a.height;
        g[r] = in ? gin[(int64_t)y * a.pitch + gx] : T(0);
    }
    // codes of the k steps (words where the region is inside the image and
    // aligned, else bytes; outside the image: CODE_NONE)
    const bool inside = rx0 >= 0 && ry0 >= 0 && rx0 + GB_RW <= a.width && ry0 + RH <= a.height &&
                        (a.width & 3) == 0 && (((uintptr_t)codes + rx0) & 3) == 0 && (a.codes_step & 3) == 0;
    if (inside) {
        constexpr int WPR = GB_RW / 4;
        for (int i = threadIdx.x; i < k * RH * WPR; i += G::THREADS) {
            const int s = i / (RH * WPR), rem = i % (RH * WPR);
            const int ly = rem / WPR, lw = rem % WPR;
            *reinterpret_cast<uint32_t *>(&scd[s][ly][4 * lw]) = *reinterpret_cast<const uint32_t *>(
                codes + s * a.codes_step + (int64_t)(ry0 + ly) * a.width + rx0 + 4 * lw);
        }
    } else {
        for (int i = threadIdx.x; i < k * RH * GB_RW; i += G::THREADS) {
            const int s = i / (RH * GB_RW), rem = i % (RH * GB_RW);
            const int ly = rem / GB_RW, lx = rem % GB_RW;
            const int y = ry0 + ly, xx = rx0 + lx;
            const bool in = (unsigned)y < (unsigned)a.height && (unsigned)xx < (unsigned)a.width;
            scd[s][ly][lx] = in ? codes[s * a.codes_step + (int64_t)y * a.width + xx] : CODE_NONE;
        }
    }
    // Mask-gradient accumulators of the lane's rows, starting from the
    // stored value so the additions keep the one-step-at-a-time order.
    const bool col_core = (unsigned)(x - GB_K) < (unsigned)GB_CX && xin;
    T acc[GB_WR];
#pragma unroll
    for (int r = 0; r < GB_WR; ++r) {
        const int ly = w * GB_WR + r, y = ry0 + ly;
        const bool in = col_core && (unsigned)(ly - GB_K) < (unsigned)CY && y < a.height;
        acc[r] = in ? gm[(int64_t)y * a.pitch + gx] : T(0);
    }
    __syncthreads();

    for (int s = k - 1; s >= 0; --s) {
        const int par = s & 1;
        // as forward: rows within s of the core still matter
        const bool busy = gb_wave_busy<CY>(w, k, k - 1 - s);
        if (busy) {
            xg[par][w][0][x] = g[0];
            xg[par][w][1][x] = g[GB_WR - 1];
        }
        __syncthreads();
        if (busy) {
            const T ga = xg[par][wa][1][x], gb = xg[par][wb][0][x];
            const int base = w * GB_WR;
            // codes and gradients of the rows around row r, columns x-1, x, x+1
            auto code_row = [&](int ly, int *c) {
                c[1] = scd[s][ly][x];
                c[0] = gb_shift<DPP_WAVE_SHR1>(c[1]);
                c[2] = gb_shift<DPP_WAVE_SHL1>(c[1]);
            };
            auto grad_row = [&](T gc, T *gr) {
                gr[1] = gc;
                gr[0] = gb_shift<DPP_WAVE_SHR1>(gc);
                gr[2] = gb_shift<DPP_WAVE_SHL1>(gc);
            };
            int c0[3], c1[3], c2[3];
            T g0[3], g1[3], g2[3];
            code_row(base > 0 ? base - 1 : RH - 1, c0);
            grad_row(ga, g0);
            code_row(base, c1);
            grad_row(g[0], g1);
            T ng[GB_WR];
#pragma unroll
            for (int r = 0; r < GB_WR; ++r) {
                code_row(base + r + 1 < RH ? base + r + 1 : 0, c2);
                grad_row(r == GB_WR - 1 ? gb : g[r + 1], g2);
                // neighbour p = q + d, d in raster order j, sent to q iff its
                // code is 8 - j
                T sum = T(0);
#pragma unroll
                for (int d = 0; d < 3; ++d)
                    if (c0[d] == 8 - d) sum += g0[d];
#pragma unroll
                for (int d = 0; d < 3; ++d)
                    if (c1[d] == 5 - d) sum += g1[d];
#pragma unroll
                for (int d = 0; d < 3; ++d)
                    if (c2[d] == 2 - d) sum += g2[d];
                ng[r] = sum;
                if (c1[1] == CODE_MASK) acc[r] += g1[1];
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    c0[d] = c1[d]; g0[d] = g1[d];
                    c1[d] = c2[d]; g1[d] = g2[d];
                }
            }
#pragma unroll
            for (int r = 0; r < GB_WR; ++r) g[r] = ng[r];
        }
    }
    // gradient w.r.t. the state before the block, and the mask gradient
#pragma unroll
    for (int r = 0; r < GB_WR; ++r) {
        const int ly = w * GB_WR + r, y = ry0 + ly;
        if (col_core && (unsigned)(ly - GB_K) < (unsigned)CY && y < a.height) {
            gout[(int64_t)y * a.pitch + gx] = g[r];
            gm[(int64_t)y * a.pitch + gx] = acc[r];
        }
    }
}

// ---------------------------------------------------------------------------
// Source tracking: the per-step routes composed over a run of steps.
//
// Following the codes backward from a pixel p of the state after step n
// (its code at step n-1, then the code of the pixel that names, ...) ends
// either at a pixel of the state before step 0, or at a step where the
// mask won, i.e. at the mask value of some pixel.  That end is p's source:
// p's value is a copy of it, and the gradient of sum(g * out) reaches that
// leaf with exactly g(p) through every step's route.  So the marker and
// mask gradients of n steps are
//   grad_marker[r] = sum of g(p) over the p whose source is marker pixel r,
//   grad_mask[r]   = sum of g(p) over the p whose source is mask pixel r,
// the same sums the step-by-step reverse pass forms, added in another order.
//
// block_src_kernel runs up to GB_K steps like block_codes_kernel, carrying
// with every pixel the id of its source: the element offset of the leaf in
// its image (y * pitch + x), with SRC_MASK set for a mask leaf.  It takes
// the same choices as the codes (the first extremal neighbour in raster
// order, the mask winning ties).  Ids of the state before the first step
// are the pixels' own offsets (ids_in == null), or those a previous launch
// wrote.  src_scatter_kernel adds g(p) to the leaf its id names.
// ---------------------------------------------------------------------------
constexpr uint32_t SRC_MASK = 0x80000000u;

struct SrcBlockArgs {
    const void *src;          // state before the block
    const void *mask;
    void *dst;                // state after the block (core pixels)
    const uint32_t *ids_in;   // ids of src, or null: each pixel its own offset
    uint32_t *ids_out;        // ids of dst
    int64_t image_stride;     // elements between images (values and ids alike)
    int64_t pitch;            // elements between rows (values and ids alike)
    int32_t width, height;
    int32_t k;                // steps in this launch (<= GB_K)
};

// Selects of ids: two unconditional selects (the compiler turns a nested
// conditional of this shape into divergent branches).
__device__ __forceinline__ uint32_t pick_id(bool first, uint32_t a, bool second, uint32_t b, uint32_t c) {
    const uint32_t t = second ? b : c;
    return first ? a : t;
}

template <typename T, int OP>
__global__ __launch_bounds__(GradTile<T>::THREADS) void block_src_kernel(SrcBlockArgs a) {
    using B = Bounds<T, OP>;
    using G = GradTile<T>;
    constexpr int CY = G::CY, NW = G::NW;
    __shared__ T xv[2][NW][2][GB_RW];          // edge rows' row-pass values
    __shared__ uint32_t xs[2][NW][2][GB_RW];   // and their source ids
    const GradBlock blk = grad_block();
    const int img = blk.img;
    const T *src = static_cast<const T *>(a.src) + img * a.image_stride;
    const T *msk = static_cast<const T *>(a.mask) + img * a.image_stride;
    T *dst = static_cast<T *>(a.dst) + img * a.image_stride;
    const uint32_t *ids_in = a.ids_in ? a.ids_in + img * a.image_stride : nullptr;
    uint32_t *ids_out = a.ids_out + img * a.image_stride;
    const int x0 = blk.bx * GB_CX, y0 = blk.by * CY;  // core origin
    const int rx0 = x0 - GB_K, ry0 = y0 - GB_K;        // region origin
    const int x = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wa = w > 0 ? w - 1 : NW - 1, wb = w < NW - 1 ? w + 1 : 0;  // region edge: harmless wrap
    const int gx = rx0 + x;
    const bool xin = (unsigned)gx < (unsigned)a.width;
    const bool col_core = (unsigned)(x - GB_K) < (unsigned)GB_CX;

    T v[GB_WR], m[GB_WR];
    uint32_t id[GB_WR], mid[GB_WR];
    // a region inside the image (most tiles) loads without per-pixel tests
    const bool interior = rx0 >= 0 && ry0 >= 0 && rx0 + GB_RW <= a.width && ry0 + NW * GB_WR <= a.height;
    if (interior) {
        const int64_t off0 = (int64_t)(ry0 + w * GB_WR) * a.pitch + gx;
#pragma unroll
        for (int r = 0; r < GB_WR; ++r) {
            const int64_t off = off0 + r * a.pitch;
            v[r] = src[off];
            m[r] = msk[off];
            id[r] = ids_in ? ids_in[off] : (uint32_t)off;
            mid[r] = SRC_MASK | (uint32_t)off;
        }
    } else {
#pragma unroll
        for (int r = 0; r < GB_WR; ++r) {
            const int y = ry0 + w * GB_WR + r;
            const bool in = xin && (unsigned)y < (unsigned)a.height;
            const int64_t off = (int64_t)y * a.pitch + gx;
            v[r] = in ? src[off] : B::bottom();
            m[r] = in ? msk[off] : B::bottom();
            // outside the image: never chosen (its value never wins), any id
            id[r] = in ? (ids_in ? ids_in[off] : (uint32_t)off) : 0u;
            mid[r] = SRC_MASK | (uint32_t)off;   // the id of this pixel's mask value
        }
    }

    // This wave's exchange slots: the parity and the edge row are compile-time
    // offsets from these (two steps per loop iteration), so the step loop
    // spends no VALU on LDS addresses.
    T *const xw = &xv[0][w][0][x];
    uint32_t *const sw = &xs[0][w][0][x];
    const T *const xa = &xv[0][wa][1][x];
    const T *const xb = &xv[0][wb][0][x];
    const uint32_t *const sa_p = &xs[0][wa][1][x];
    const uint32_t *const sb_p = &xs[0][wb][0][x];
    constexpr int PAR_T = NW * 2 * GB_RW;   // elements between the parities
    constexpr int ROW_T = GB_RW;            // between a wave's first and last row

    const int k = a.k;
    // row-pass results of a step (kept across steps: a wave that skips a
    // step neither writes nor reads them)
    T h[GB_WR];
    uint32_t hs[GB_WR];
    auto step = [&](int s, auto par_tag) {
        constexpr int par = decltype(par_tag)::value;
        const bool busy = gb_wave_busy<CY>(w, k, s);
        if (busy) {
            // row pass: the first of (x-1, x, x+1) equal to their extremum
#pragma unroll
            for (int r = 0; r < GB_WR; ++r) {
                const T c = v[r];
                const T left = gb_shift<DPP_WAVE_SHR1>(c);
                const T right = gb_shift<DPP_WAVE_SHL1>(c);
                const uint32_t il = (uint32_t)gb_shift<DPP_WAVE_SHR1>((int)id[r]);
                const uint32_t ir = (uint32_t)gb_shift<DPP_WAVE_SHL1>((int)id[r]);
                const T best = extremum<OP>(extremum<OP>(left, c), right);
                h[r] = best;
                hs[r] = pick_id(left == best, il, c == best, id[r], ir);
            }
            xw[par * PAR_T] = h[0];
            sw[par * PAR_T] = hs[0];
            xw[par * PAR_T + ROW_T] = h[GB_WR - 1];
            sw[par * PAR_T + ROW_T] = hs[GB_WR - 1];
        }
        __syncthreads();
        if (busy) {
            const T ha = xa[par * PAR_T], hb = xb[par * PAR_T];
            const uint32_t sa = sa_p[par * PAR_T], sb = sb_p[par * PAR_T];
            // column pass (rows y-1, y, y+1 in that order), then the clamp
            // (the mask wins ties); the row pass results are all read before
            // v and id are overwritten
#pragma unroll
            for (int r = 0; r < GB_WR; ++r) {
                const T hu = r == 0 ? ha : h[r - 1];
                const uint32_t su = r == 0 ? sa : hs[r - 1];
                const T hd = r == GB_WR - 1 ? hb : h[r + 1];
                const uint32_t sd = r == GB_WR - 1 ? sb : hs[r + 1];
                const T best = extremum<OP>(extremum<OP>(hu, h[r]), hd);
                const uint32_t from = pick_id(hu == best, su, h[r] == best, hs[r], sd);
                const bool mask_wins = OP == OP_DILATE ? !(best < m[r]) : !(best > m[r]);
                v[r] = mask_wins ? m[r] : best;
                id[r] = mask_wins ? mid[r] : from;
            }
        }
    };
    for (int s = 0; s < k; s += 2) {
        step(s, std::integral_constant<int, 0>{});
        if (s + 1 < k) step(s + 1, std::integral_constant<int, 1>{});
    }
    // core of the state after the block, with its ids
    if (col_core && xin) {
#pragma unroll
        for (int r = 0; r < GB_WR; ++r) {
            const int ly = w * GB_WR + r, y = ry0 + ly;
            if ((unsigned)(ly - GB_K) < (unsigned)CY && y < a.height) {
                const int64_t off = (int64_t)y * a.pitch + gx;
                dst[off] = v[r];
                ids_out[off] = id[r];
            }
        }
    }
}

struct SrcScatterArgs {
    const uint32_t *ids;      // source of every pixel of the state after the run
    const void *g_out;        // upstream gradient (that state's gradient)
    void *g_marker;           // gradient of the state before the run: zero on entry
    void *g_mask;             // mask gradient, accumulated
    int64_t image_stride, pitch;
    int32_t width, height, n_images;
    uint32_t span;            // elements of one image, (height - 1) * pitch + width
};

// The scatter in two passes.  Pass 1 (src_local_kernel) streams over the
// pixels: the marker gradient of pixel p becomes g(p) if p's source is its
// own marker pixel and 0 otherwise, and the mask gradient of p gains g(p)
// if p's source is its own mask pixel; no other pixel of the pass writes
// there, so these are plain accesses.  Pass 2 (src_scatter_kernel), after
// it, adds the gradient of every other pixel to the leaf its id names with
// hardware atomics.  In the chains of a reconstruction most pixels end as
// copies of their own mask value, so pass 2 has little to do.  Additions
// into one leaf from several pixels come in no fixed order, so results may
// differ between runs in the last bits.
// Grid: x over the columns of a row, y over rows (strided), z = image.
template <typename T>
__global__ void src_local_kernel(SrcScatterArgs a) {
    const int64_t base = (int64_t)blockIdx.z * a.image_stride;
    const T *g = static_cast<const T *>(a.g_out) + base;
    T *gf = static_cast<T *>(a.g_marker) + base;
    T *gm = static_cast<T *>(a.g_mask) + base;
    const uint32_t *ids = a.ids + base;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= a.width) return;
    for (int y = blockIdx.y; y < a.height; y += gridDim.y) {
        const uint32_t pos = (uint32_t)((int64_t)y * a.pitch + x);
        const uint32_t id = ids[pos];
        const T gv = g[pos];
        gf[pos] = id == pos ? gv : T(0);
        if (id == (SRC_MASK | pos) && gv != T(0)) gm[pos] += gv;
    }
}

template <typename T>
__global__ void src_scatter_kernel(SrcScatterArgs a) {
    const int64_t base = (int64_t)blockIdx.z * a.image_stride;
    const T *g = static_cast<const T *>(a.g_out) + base;
    T *gf = static_cast<T *>(a.g_marker) + base;
    T *gm = static_cast<T *>(a.g_mask) + base;
    const uint32_t *ids = a.ids + base;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= a.width) return;
    for (int y = blockIdx.y; y < a.height; y += gridDim.y) {
        const uint32_t pos = (uint32_t)((int64_t)y * a.pitch + x);
        const uint32_t id = ids[pos];
        const uint32_t leaf = id & ~SRC_MASK;
        if (leaf == pos) continue;      // own pixel: pass 1
        if (leaf >= a.span) continue;   // not an element of the image: ignored
        const T gv = g[pos];
        if (gv == T(0)) continue;
        unsafeAtomicAdd((id & SRC_MASK) ? gm + leaf : gf + leaf, gv);
    }
}

}  // namespace geochain
