// window_hgw.hpp -- size-insensitive path for plain chains: n elementary 3x3
// dilations (erosions) equal one (2n+1) x (2n+1) window maximum (minimum)
// clipped to the image (Eq. 1-2, 4), and that window decomposes into a row
// window and a column window of 2n+1 (Section 3.1).  Each 1-D window is
// computed with the van Herk / Gil-Werman prefix-suffix scheme cited in the
// introduction: the line, padded by n neutral values at each end, is cut
// into blocks of w = 2n+1; with g = the running extremum from the start of
// each block and h = the running extremum to its end, the window starting at
// padded position s is exactly pick(h[s], g[s + 2n]) -- a cost per pixel
// that does not depend on n.
//
// hgw_rows_kernel: one wave per line, lanes along the line.  Each 64-pixel
// chunk runs a segmented inclusive scan with DPP (row_shr 1, 2, 4, 8 inside
// 16-lane rows, then row_bcast 15 and 31 across rows; a lane takes a partner
// only if the partner lies in its block) and a carry from the previous
// chunk.  The line is first staged in LDS (its loads all in flight at
// once); the forward sweep stores g in LDS; the backward sweep reads each
// chunk in reversed lane order, so the same prefix scan yields h, and emits
// the outputs of that chunk at once.  Columns go through the same kernel
// between two tiled transposes (transpose_kernel, 64 x 64 tiles in LDS).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "chain_block.hpp"

namespace geochain {

struct HgwArgs {
    const void *src;
    void *dst;
    int32_t length;      // pixels per line
    int32_t lines;
    int64_t src_pitch;   // elements between line starts
    int64_t dst_pitch;
    int32_t n;           // window radius along the line, 0 <= n < length
    int32_t chunks;      // ceil((length + 2n) / 64)
};

// DPP move of a register value; lanes that receive nothing keep `old`.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t hgw_dpp(uint32_t old, uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, CTRL, ROW_MASK, 0xF, false);
}
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float hgw_dpp(float old, float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, old),
                                                                 __builtin_bit_cast(int, v), CTRL, ROW_MASK, 0xF,
                                                                 false));
}
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double hgw_dpp(double old, double v) {
    const uint64_t o = __builtin_bit_cast(uint64_t, old), u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)o, (int)(uint32_t)u, CTRL, ROW_MASK,
                                                              0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)(o >> 32), (int)(uint32_t)(u >> 32),
                                                              CTRL, ROW_MASK, 0xF, false);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ uint32_t hgw_lane63(uint32_t v) { return (uint32_t)__builtin_amdgcn_readlane((int)v, 63); }
__device__ __forceinline__ float hgw_lane63(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}
__device__ __forceinline__ double hgw_lane63(double v) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, 63);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), 63);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Inclusive scan of pick over lanes 0..l restricted to the lanes of l's
// block: o = how many lanes before l (in lane order) belong to its block,
// capped by nothing (values >= 64 mean "all of them").
template <int OP, typename R>
__device__ __forceinline__ R hgw_segmented_scan(R v, int o, int lane) {
    using P = Pick<OP>;
    const R id = Bounds<R, OP>::bottom();
    R t;
    t = hgw_dpp<0x111, 0xF>(id, v);  // row_shr:1
    v = o >= 1 ? P::pick(v, t) : v;
    t = hgw_dpp<0x112, 0xF>(id, v);  // row_shr:2
    v = o >= 2 ? P::pick(v, t) : v;
    t = hgw_dpp<0x114, 0xF>(id, v);  // row_shr:4
    v = o >= 4 ? P::pick(v, t) : v;
    t = hgw_dpp<0x118, 0xF>(id, v);  // row_shr:8
    v = o >= 8 ? P::pick(v, t) : v;
    // lane 15 of row r -> every lane of row r + 1 (rows 1 and 3)
    t = hgw_dpp<0x142, 0xA>(id, v);  // row_bcast:15
    v = o > (lane & 15) && (lane & 16) ? P::pick(v, t) : v;
    // lane 31 -> every lane of rows 2 and 3
    t = hgw_dpp<0x143, 0xC>(id, v);  // row_bcast:31
    v = o > (lane & 31) && (lane & 32) ? P::pick(v, t) : v;
    return v;
}

template <typename T, int OP>
__global__ __launch_bounds__(64) void hgw_rows_kernel(HgwArgs a) {
    using R = typename RegOf<T>::type;
    using P = Pick<OP>;
    extern __shared__ unsigned char hgw_lds_raw[];
    R *g = reinterpret_cast<R *>(hgw_lds_raw);                    // chunks * 64 values
    T *line_px = reinterpret_cast<T *>(g + a.chunks * 64);        // the line, `length` pixels

    const int line = blockIdx.x;
    const int lane = threadIdx.x;
    const T *src = static_cast<const T *>(a.src) + (int64_t)line * a.src_pitch;
    T *dst = static_cast<T *>(a.dst) + (int64_t)line * a.dst_pitch;
    const int n = a.n;
    const int w = 2 * n + 1;
    const R neutral = Bounds<R, OP>::bottom();

    // Stage the line in LDS: all its loads in flight at once, instead of one
    // exposed memory latency per chunk in the dependent sweeps below.
    constexpr int U = 8;
    for (int x0 = 0; x0 < a.length; x0 += 64 * U) {
        T vals[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int x = x0 + u * 64 + lane;
            vals[u] = x < a.length ? src[x] : T(0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int x = x0 + u * 64 + lane;
            if (x < a.length) line_px[x] = vals[u];
        }
    }
    __syncthreads();

    // pm = p mod w, advanced by 64 per chunk without a division when w > 64
    auto step_mod = [&](int pm, int delta) {
        if (w > 64) {
            pm += delta;
            return pm >= w ? pm - w : (pm < 0 ? pm + w : pm);
        }
        return ((pm + delta) % w + w) % w;
    };

    // forward sweep: g (running extremum from each block's start)
    R carry = neutral;
    int pm = lane % w;
    for (int c = 0; c < a.chunks; ++c) {
        const int p = c * 64 + lane;            // padded position
        const int x = p - n;
        const R v = (unsigned)x < (unsigned)a.length ? to_reg(line_px[x]) : neutral;
        R s = hgw_segmented_scan<OP>(v, pm, lane);   // pm = block lanes before p
        s = pm > lane ? P::pick(s, carry) : s;       // block started in an earlier chunk
        g[p] = s;
        carry = hgw_lane63(s);
        pm = step_mod(pm, 64);
    }
    __syncthreads();

    // backward sweep in reversed lane order: h (running extremum to each
    // block's end), and the outputs pick(h[s], g[s + 2n]) for s < length.
    carry = neutral;
    pm = ((a.chunks - 1) * 64 + 63 - lane) % w;
    for (int c = a.chunks - 1; c >= 0; --c) {
        const int p = c * 64 + 63 - lane;
        const int x = p - n;
        const R v = (unsigned)x < (unsigned)a.length ? to_reg(line_px[x]) : neutral;
        const int o = w - 1 - pm;               // block lanes after p
        R s = hgw_segmented_scan<OP>(v, o, lane);
        s = o > lane ? P::pick(s, carry) : s;
        carry = hgw_lane63(s);
        if (p < a.length) from_reg(dst + p, P::pick(s, g[p + 2 * n]));
        pm = step_mod(pm, -64);
    }
}

// dst (H x W, row = source column) = transpose of src (W x H).
template <typename T>
__global__ __launch_bounds__(256) void transpose_kernel(const T *src, T *dst, int32_t width, int32_t height,
                                                        int64_t src_pitch, int64_t dst_pitch) {
    __shared__ T tile[64][65];
    const int bx = blockIdx.x * 64, by = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;   // 64 x 4 threads
    for (int r = ty; r < 64; r += 4) {
        const int x = bx + tx, y = by + r;
        if (x < width && y < height) tile[r][tx] = src[(int64_t)y * src_pitch + x];
    }
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {
        const int y = by + tx, x = bx + r;   // dst row x, column y
        if (x < width && y < height) dst[(int64_t)x * dst_pitch + y] = tile[tx][r];
    }
}

}  // namespace geochain
