// grad_step.hpp -- kernels for differentiating a geodesic chain (not part of
// the paper, which has no backward pass).
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
// decomposes as in Section 3.1).
//
// The backward kernel is a GATHER: pixel q collects the upstream gradient of
// every neighbour p whose code points at q, visiting p in raster order, and
// the mask gradient collects g(q) where code(q) == 9.  One launch is one step
// for a whole batch of images (grid.z = image); tiles of 64 x 16 pixels with
// a one-pixel halo are staged in LDS so each value is read once per tile.
//
// Values must be finite: a pixel outside the image is represented by the
// neutral extremum (-inf for dilation), which must never tie with a real
// value.  Codes are stored densely: codes[image][step][y][width] bytes.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "chain_block.hpp"

namespace geochain {

constexpr int GT_X = 64;   // tile width
constexpr int GT_Y = 16;   // tile height
constexpr int GT_THREADS = 256;
constexpr uint8_t CODE_MASK = 9;
constexpr uint8_t CODE_NONE = 255;

struct StepArgs {
    const void *src;      // state before the step
    const void *mask;
    void *dst;            // state after the step
    uint8_t *codes;       // codes of this step (image 0); next image at +codes_image_stride
    int64_t codes_image_stride;
    int64_t image_stride; // elements between images of src / mask / dst
    int64_t pitch;
    int32_t width, height;
};

struct BwdArgs {
    const uint8_t *codes; // codes of this step (image 0)
    int64_t codes_image_stride;
    const void *g_in;     // gradient w.r.t. the step's output
    void *g_out;          // gradient w.r.t. the step's input (written)
    void *g_mask;         // gradient w.r.t. the mask (accumulated)
    int64_t image_stride;
    int64_t pitch;
    int32_t width, height;
};

template <int OP, typename T>
__device__ __forceinline__ bool better(T a, T b) {
    return OP == OP_DILATE ? (a > b) : (a < b);
}

template <typename T, int OP>
__global__ __launch_bounds__(GT_THREADS) void step_codes_kernel(StepArgs a) {
    using B = Bounds<T, OP>;
    __shared__ T s[GT_Y + 2][GT_X + 2];
    const int img = blockIdx.z;
    const T *src = static_cast<const T *>(a.src) + img * a.image_stride;
    const T *msk = static_cast<const T *>(a.mask) + img * a.image_stride;
    T *dst = static_cast<T *>(a.dst) + img * a.image_stride;
    uint8_t *codes = a.codes + img * a.codes_image_stride;
    const int x0 = blockIdx.x * GT_X, y0 = blockIdx.y * GT_Y;

    for (int i = threadIdx.x; i < (GT_Y + 2) * (GT_X + 2); i += GT_THREADS) {
        const int ly = i / (GT_X + 2), lx = i % (GT_X + 2);
        const int y = y0 + ly - 1, x = x0 + lx - 1;
        const bool in = (unsigned)y < (unsigned)a.height && (unsigned)x < (unsigned)a.width;
        s[ly][lx] = in ? src[(int64_t)y * a.pitch + x] : B::bottom();
    }
    __syncthreads();

    const int lx = threadIdx.x % GT_X;
    for (int ly = threadIdx.x / GT_X; ly < GT_Y; ly += GT_THREADS / GT_X) {
        const int x = x0 + lx, y = y0 + ly;
        if (x >= a.width || y >= a.height) continue;
        // row pass with the earliest extremum of each row, then column pass
        T best = B::bottom();
        int code = -1;
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
            T rv = s[ly + dy][lx];
            int rdx = 0;
            const T c = s[ly + dy][lx + 1], r = s[ly + dy][lx + 2];
            if (better<OP>(c, rv)) { rv = c; rdx = 1; }
            if (better<OP>(r, rv)) { rv = r; rdx = 2; }
            if (code < 0 || better<OP>(rv, best)) { best = rv; code = dy * 3 + rdx; }
        }
        const int64_t off = (int64_t)y * a.pitch + x;
        const T m = msk[off];
        const bool mask_wins = OP == OP_DILATE ? !(best < m) : !(best > m);
        dst[off] = mask_wins ? m : best;
        codes[(int64_t)y * a.width + x] = mask_wins ? CODE_MASK : (uint8_t)code;
    }
}

template <typename T>
__global__ __launch_bounds__(GT_THREADS) void step_bwd_kernel(BwdArgs a) {
    __shared__ T sg[GT_Y + 2][GT_X + 2];
    __shared__ uint8_t sc[GT_Y + 2][GT_X + 2];
    const int img = blockIdx.z;
    const T *gin = static_cast<const T *>(a.g_in) + img * a.image_stride;
    T *gout = static_cast<T *>(a.g_out) + img * a.image_stride;
    T *gm = static_cast<T *>(a.g_mask) + img * a.image_stride;
    const uint8_t *codes = a.codes + img * a.codes_image_stride;
    const int x0 = blockIdx.x * GT_X, y0 = blockIdx.y * GT_Y;

    for (int i = threadIdx.x; i < (GT_Y + 2) * (GT_X + 2); i += GT_THREADS) {
        const int ly = i / (GT_X + 2), lx = i % (GT_X + 2);
        const int y = y0 + ly - 1, x = x0 + lx - 1;
        const bool in = (unsigned)y < (unsigned)a.height && (unsigned)x < (unsigned)a.width;
        sg[ly][lx] = in ? gin[(int64_t)y * a.pitch + x] : T(0);
        sc[ly][lx] = in ? codes[(int64_t)y * a.width + x] : CODE_NONE;
    }
    __syncthreads();

    const int lx = threadIdx.x % GT_X;
    for (int ly = threadIdx.x / GT_X; ly < GT_Y; ly += GT_THREADS / GT_X) {
        const int x = x0 + lx, y = y0 + ly;
        if (x >= a.width || y >= a.height) continue;
        // Neighbour p = q + d (d in raster order j = 0..8) sent its gradient
        // to q iff its code names the offset q - p = -d, i.e. code 8 - j.
        T acc = T(0);
#pragma unroll
        for (int j = 0; j < 9; ++j) {
            const int dy = j / 3, dx = j % 3;
            if (sc[ly + dy][lx + dx] == 8 - j) acc += sg[ly + dy][lx + dx];
        }
        const int64_t off = (int64_t)y * a.pitch + x;
        gout[off] = acc;
        if (sc[ly + 1][lx + 1] == CODE_MASK) gm[off] += sg[ly + 1][lx + 1];
    }
}

}  // namespace geochain
