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
// hgw_rows_kernel: one wave per line.  The line is staged in LDS (all its
// loads in flight at once); each lane then owns a contiguous segment of S
// padded positions (S odd, so the lanes' LDS accesses fall in distinct
// banks) and runs the running extrema through it sequentially, restarting at
// block boundaries.  A segmented scan across the 64 lanes (shuffles) gives
// each segment the extremum carried in from its neighbour, which the
// positions before the segment's first block boundary then take.  Both g
// (forward) and h (backward) are built this way in LDS, and the outputs are
// written coalesced.  Columns go through the same kernel between two tiled
// transposes (transpose_kernel, 64 x 64 tiles in LDS).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

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
    int32_t seg;         // positions per lane: odd, 64 seg >= length + 2n
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

// Segmented inclusive scan over the 64 lanes of (val, flag) pairs, in lane
// order (FORWARD: lane l combines lanes 0..l) or reversed (lanes l..63):
// a lane whose flag is set starts a new segment; otherwise it takes the
// extremum of its value and the scan of the lanes before it.
template <int OP, bool FORWARD, typename R>
__device__ __forceinline__ R hgw_lane_scan(R val, int flag) {
    using P = Pick<OP>;
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const R v2 = FORWARD ? __shfl_up(val, d) : __shfl_down(val, d);
        const int f2 = FORWARD ? __shfl_up(flag, d) : __shfl_down(flag, d);
        const bool has = FORWARD ? lane >= d : lane + d < 64;
        if (has && !flag) val = P::pick(val, v2);
        if (has) flag |= f2;
    }
    return val;
}

template <typename T, int OP>
__global__ __launch_bounds__(64) void hgw_rows_kernel(HgwArgs a) {
    using R = typename RegOf<T>::type;
    using P = Pick<OP>;
    extern __shared__ unsigned char hgw_lds_raw[];
    const int S = a.seg;                                          // positions per lane (odd)
    R *__restrict__ g = reinterpret_cast<R *>(hgw_lds_raw);       // 64 S running extrema from block starts
    R *__restrict__ h = reinterpret_cast<R *>(hgw_lds_raw) + 64 * S;   // 64 S running extrema to block ends
    T *__restrict__ line_px = reinterpret_cast<T *>(reinterpret_cast<R *>(hgw_lds_raw) + 128 * S);

    const int line = blockIdx.x;
    const int lane = threadIdx.x;
    const T *src = static_cast<const T *>(a.src) + (int64_t)line * a.src_pitch;
    T *dst = static_cast<T *>(a.dst) + (int64_t)line * a.dst_pitch;
    const int n = a.n;
    const int w = 2 * n + 1;
    const R neutral = Bounds<R, OP>::bottom();

    // Stage the line in LDS with all its loads in flight.
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
    auto padded = [&](int p) {   // the line padded by n neutral pixels each side
        const int x = p - n;
        return (unsigned)x < (unsigned)a.length ? to_reg(line_px[x]) : neutral;
    };

    // Each lane owns the padded positions [base, base + S).  Sequential
    // running extrema inside the segment, restarting at block boundaries;
    // then the lanes' segment summaries are scanned across lanes and the
    // positions of each segment that continue a block from a neighbouring
    // segment take its carry.
    const int base = lane * S;
    const int pm0 = base % w;                 // base's offset inside its block

    // forward: g
    R acc = neutral;
    int first_start = S;                      // first block start in the segment
    {
        int pm = pm0;
        for (int i = 0; i < S; ++i) {
            const R v = padded(base + i);
            const bool start = pm == 0;
            acc = start ? v : P::pick(acc, v);
            first_start = (start && first_start == S) ? i : first_start;
            g[base + i] = acc;
            pm = pm + 1 == w ? 0 : pm + 1;
        }
    }
    {
        const R scanned = hgw_lane_scan<OP, true>(acc, first_start < S ? 1 : 0);
        R carry = __shfl_up(scanned, 1);
        carry = lane == 0 ? neutral : carry;
        for (int i = 0; i < first_start; ++i) g[base + i] = P::pick(g[base + i], carry);
    }

    // backward: h
    acc = neutral;
    int last_end = -1;                        // last block end in the segment
    {
        int pm = (base + S - 1) % w;
        for (int i = S - 1; i >= 0; --i) {
            const R v = padded(base + i);
            const bool end = pm == w - 1;
            acc = end ? v : P::pick(acc, v);
            last_end = (end && last_end < 0) ? i : last_end;
            h[base + i] = acc;
            pm = pm == 0 ? w - 1 : pm - 1;
        }
    }
    {
        const R scanned = hgw_lane_scan<OP, false>(acc, last_end >= 0 ? 1 : 0);
        R carry = __shfl_down(scanned, 1);
        carry = lane == 63 ? neutral : carry;
        for (int i = S - 1; i > last_end; --i) h[base + i] = P::pick(h[base + i], carry);
    }
    __syncthreads();

    // outputs: the window starting at padded position x covers [x, x + 2n]
    for (int x = lane; x < a.length; x += 64) from_reg(dst + x, P::pick(h[x], g[x + 2 * n]));
}

// Inclusive segmented scan in lane order by DPP: a lane whose flag is set
// starts a segment; otherwise it takes the extremum of its value and the
// scan of the lanes before it.  row_shr 1, 2, 4, 8 scan each 16-lane row,
// row_bcast 15 and 31 then carry rows 0 and 0-1 into the rows after them.
template <int OP, typename R>
__device__ __forceinline__ R hgw_flag_scan(R val, int flag) {
    using P = Pick<OP>;
    const R id = Bounds<R, OP>::bottom();
    auto step = [&](auto ctrl_tag, auto mask_tag) {
        constexpr int CTRL = decltype(ctrl_tag)::value, MASK = decltype(mask_tag)::value;
        const R t = hgw_dpp<CTRL, MASK>(id, val);
        const int tf = (int)hgw_dpp<CTRL, MASK>(0u, (uint32_t)flag);
        val = flag ? val : P::pick(val, t);
        flag |= tf;
    };
    step(std::integral_constant<int, 0x111>{}, std::integral_constant<int, 0xF>{});
    step(std::integral_constant<int, 0x112>{}, std::integral_constant<int, 0xF>{});
    step(std::integral_constant<int, 0x114>{}, std::integral_constant<int, 0xF>{});
    step(std::integral_constant<int, 0x118>{}, std::integral_constant<int, 0xF>{});
    step(std::integral_constant<int, 0x142>{}, std::integral_constant<int, 0xA>{});
    step(std::integral_constant<int, 0x143>{}, std::integral_constant<int, 0xC>{});
    return val;
}

// The same line window with each lane's segment held in registers: the
// segment length S is the compile-time constant (the host pads the line to
// 64 S positions with neutral values), so every loop unrolls without guards
// and each sweep's LDS reads go out as one batch instead of one dependent
// read per position.  The backward sweep gives lane l the segment 63 - l, so
// its scan across lanes also runs in lane order.
template <typename T, int OP, int S>
__global__ __launch_bounds__(64) void hgw_rows_reg_kernel(HgwArgs a) {
    using R = typename RegOf<T>::type;
    using P = Pick<OP>;
    extern __shared__ unsigned char hgw_lds_raw[];
    R *__restrict__ g = reinterpret_cast<R *>(hgw_lds_raw);
    R *__restrict__ h = reinterpret_cast<R *>(hgw_lds_raw) + 64 * S;
    T *__restrict__ line_px = reinterpret_cast<T *>(reinterpret_cast<R *>(hgw_lds_raw) + 128 * S);

    const int line = blockIdx.x;
    const int lane = threadIdx.x;
    const T *src = static_cast<const T *>(a.src) + (int64_t)line * a.src_pitch;
    T *dst = static_cast<T *>(a.dst) + (int64_t)line * a.dst_pitch;
    const int n = a.n;
    const int w = 2 * n + 1;
    const R neutral = Bounds<R, OP>::bottom();

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
    auto padded = [&](int p) {
        const int x = p - n;
        return (unsigned)x < (unsigned)a.length ? to_reg(line_px[x]) : neutral;
    };

    // forward: lane l owns segment l
    {
        const int base = lane * S;
        R v[S];
#pragma unroll
        for (int i = 0; i < S; ++i) v[i] = padded(base + i);
        R acc = neutral;
        int first_start = S;
        int pm = base % w;
#pragma unroll
        for (int i = 0; i < S; ++i) {
            const bool start = pm == 0;
            acc = start ? v[i] : P::pick(acc, v[i]);
            first_start = (start && first_start == S) ? i : first_start;
            v[i] = acc;
            pm = pm + 1 == w ? 0 : pm + 1;
        }
        const R scanned = hgw_flag_scan<OP>(acc, first_start < S ? 1 : 0);
        const R carry = hgw_dpp<DPP_WAVE_SHR1, 0xF>(neutral, scanned);   // lane l - 1's, lane 0: neutral
#pragma unroll
        for (int i = 0; i < S; ++i) g[base + i] = i < first_start ? P::pick(v[i], carry) : v[i];
    }
    // backward: lane l owns segment 63 - l, scanned from its end
    {
        const int base = (63 - lane) * S;
        R v[S];
#pragma unroll
        for (int i = 0; i < S; ++i) v[i] = padded(base + i);
        R acc = neutral;
        int last_end = -1;
        int pm = (base + S - 1) % w;
#pragma unroll
        for (int i = S - 1; i >= 0; --i) {
            const bool end = pm == w - 1;
            acc = end ? v[i] : P::pick(acc, v[i]);
            last_end = (end && last_end < 0) ? i : last_end;
            v[i] = acc;
            pm = pm == 0 ? w - 1 : pm - 1;
        }
        const R scanned = hgw_flag_scan<OP>(acc, last_end >= 0 ? 1 : 0);
        const R carry = hgw_dpp<DPP_WAVE_SHR1, 0xF>(neutral, scanned);   // the segment to the right
#pragma unroll
        for (int i = 0; i < S; ++i) h[base + i] = i > last_end ? P::pick(v[i], carry) : v[i];
    }
    __syncthreads();
    for (int x = lane; x < a.length; x += 64) from_reg(dst + x, P::pick(h[x], g[x + 2 * n]));
}

// dst (H x W, row = source column) = transpose of src (W x H), 64 x 64
// tiles through LDS.  VEC: every row start of both images is 16-byte
// aligned, so each thread moves 16 bytes per global access (one tile row of
// 64 u8, or a quarter / eighth of an f32 / f64 row); otherwise one element.
template <typename T, bool VEC>
__global__ __launch_bounds__(256) void transpose_kernel(const T *__restrict__ src, T *__restrict__ dst, int32_t width,
                                                        int32_t height, int64_t src_pitch, int64_t dst_pitch) {
    constexpr int TILE = 64;
    constexpr int PAD = 16 / (int)sizeof(T) > 1 ? 16 / (int)sizeof(T) : 1;
    __shared__ T tile[TILE][TILE + PAD];
    const int bx = blockIdx.x * TILE, by = blockIdx.y * TILE;
    if constexpr (VEC) {
        constexpr int V = 16 / (int)sizeof(T);         // elements per 16 bytes
        constexpr int TPR = TILE / V;                   // threads per tile row
        constexpr int RPI = 256 / TPR;                  // tile rows per iteration
        const int c0 = (threadIdx.x % TPR) * V;
        for (int r = threadIdx.x / TPR; r < TILE; r += RPI) {
            const int y = by + r, x = bx + c0;
            if (y < height && x + V <= width) {
                union { uint4 v; T e[V]; } u;
                u.v = *reinterpret_cast<const uint4 *>(src + (int64_t)y * src_pitch + x);
#pragma unroll
                for (int j = 0; j < V; ++j) tile[r][c0 + j] = u.e[j];
            } else if (y < height) {
                for (int j = 0; j < V && x + j < width; ++j) tile[r][c0 + j] = src[(int64_t)y * src_pitch + x + j];
            }
        }
        __syncthreads();
        // dst row = source column bx + r; its elements by .. by + 63
        for (int r = threadIdx.x / TPR; r < TILE; r += RPI) {
            const int x = bx + r, y = by + c0;
            if (x >= width) continue;
            if (y + V <= height) {
                union { uint4 v; T e[V]; } u;
#pragma unroll
                for (int j = 0; j < V; ++j) u.e[j] = tile[c0 + j][r];
                *reinterpret_cast<uint4 *>(dst + (int64_t)x * dst_pitch + y) = u.v;
            } else {
                for (int j = 0; j < V && y + j < height; ++j) dst[(int64_t)x * dst_pitch + y + j] = tile[c0 + j][r];
            }
        }
    } else {
        const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;   // 64 x 4 threads
        for (int r = ty; r < TILE; r += 4) {
            const int x = bx + tx, y = by + r;
            if (x < width && y < height) tile[r][tx] = src[(int64_t)y * src_pitch + x];
        }
        __syncthreads();
        for (int r = ty; r < TILE; r += 4) {
            const int y = by + tx, x = bx + r;
            if (x < width && y < height) dst[(int64_t)x * dst_pitch + y] = tile[tx][r];
        }
    }
}

}  // namespace geochain
