// chain_block.hpp -- temporal-blocked kernel for chains of elementary 3x3
// geodesic (or plain) dilations / erosions on gfx950.
//
// One launch advances the image by k steps (Eq. 4 iterated k times).  Each
// workgroup owns an output tile ("core") and loads the core plus a k-pixel
// halo ("region") into REGISTERS.  It then runs k steps entirely on chip and
// writes the core back.  Pixels near the region's outer edge see wrong
// neighbours, but an error travels one pixel per step, so after k steps the
// core is still exact.  This replaces the paper's CPU pipeline of in-place
// streaming filters (Section 3.3-3.5): on the GPU the halo recomputation buys
// k steps per trip to memory instead of one.
//
// Register layout (per workgroup of NW waves):
//   region = (64*CW) columns x (NW*RPW) rows;
//   wave w owns rows [w*RPW, (w+1)*RPW) of the region;
//   lane l of a wave owns columns [l*CW, (l+1)*CW) of those rows.
//
// One step (Section 3.1: the 3x3 square decomposes into a 1x3 row pass and
// a 3x1 column pass, 4 comparisons per pixel; Section 3.4 keeps the row-pass
// results of neighbouring rows so each is computed once):
//   1. row pass: h = extremum of (left, centre, right); the neighbour columns
//      of the lane's edge pixels come from the adjacent lanes through DPP
//      wave shifts (no memory traffic);
//   2. the row-pass results of each wave's first and last rows go through
//      LDS to the waves above and below (one barrier per step);
//   3. column pass over the three row-pass results, then the geodesic clamp
//      against the mask held in registers (Eq. 3).
//
// Image borders: pixels of the region outside the image hold the neutral
// value (bottom for dilation, top for erosion) and a neutral mask, so the
// clamp pins them to neutral every step; a neutral value never wins the
// window extremum, which is exactly the clipped window of Section 2.
//
// Reconstruction (Eq. 5): for every step, each wave ORs "some core pixel
// changed" into a per-launch bit mask (bit s = step s changed something),
// which becomes a global word by one atomic OR per wave.  A launch whose
// predecessor's word is not all-ones (the image had stopped changing)
// exits at once; this is the GPU counterpart of the convergence flag of
// Section 3.7.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace geochain {

enum : int { OP_DILATE = 0, OP_ERODE = 1 };

// Kernel mode: where the clamp mask comes from.
enum : int {
    MODE_GEODESIC = 0,   // mask read from memory (Eq. 3)
    MODE_PLAIN = 1,      // no mask (Eq. 1-2); the clamp only fences the border
    MODE_MIXED = 2,      // as MODE_PLAIN, each step a dilation or an erosion
                         // (BlockArgs::erode_bits; one lane group per wave;
                         // launched for u8 and f32)
};

template <typename T> struct RegOf;
template <> struct RegOf<uint8_t> { using type = uint32_t; };
template <> struct RegOf<float> { using type = float; };
template <> struct RegOf<double> { using type = double; };

// bottom(OP): never wins the window extremum; top(OP): never wins the clamp.
template <typename R, int OP> struct Bounds;
template <> struct Bounds<uint32_t, OP_DILATE> {
    static __device__ __forceinline__ uint32_t bottom() { return 0u; }
    static __device__ __forceinline__ uint32_t top() { return 255u; }
};
template <> struct Bounds<uint32_t, OP_ERODE> {
    static __device__ __forceinline__ uint32_t bottom() { return 255u; }
    static __device__ __forceinline__ uint32_t top() { return 0u; }
};
template <> struct Bounds<float, OP_DILATE> {
    static __device__ __forceinline__ float bottom() { return -__builtin_inff(); }
    static __device__ __forceinline__ float top() { return __builtin_inff(); }
};
template <> struct Bounds<float, OP_ERODE> {
    static __device__ __forceinline__ float bottom() { return __builtin_inff(); }
    static __device__ __forceinline__ float top() { return -__builtin_inff(); }
};
template <> struct Bounds<double, OP_DILATE> {
    static __device__ __forceinline__ double bottom() { return -__builtin_inf(); }
    static __device__ __forceinline__ double top() { return __builtin_inf(); }
};
template <> struct Bounds<double, OP_ERODE> {
    static __device__ __forceinline__ double bottom() { return __builtin_inf(); }
    static __device__ __forceinline__ double top() { return -__builtin_inf(); }
};

// pick = the window extremum (max for dilation, min for erosion);
// clamp = the geodesic constraint (min for dilation, max for erosion).
template <int OP> struct Pick;
template <> struct Pick<OP_DILATE> {
    static __device__ __forceinline__ uint32_t pick(uint32_t a, uint32_t b) { return a > b ? a : b; }
    static __device__ __forceinline__ float pick(float a, float b) { return __builtin_fmaxf(a, b); }
    static __device__ __forceinline__ double pick(double a, double b) { return __builtin_fmax(a, b); }
    static __device__ __forceinline__ uint32_t clamp(uint32_t a, uint32_t b) { return a < b ? a : b; }
    static __device__ __forceinline__ float clamp(float a, float b) { return __builtin_fminf(a, b); }
    static __device__ __forceinline__ double clamp(double a, double b) { return __builtin_fmin(a, b); }
};
template <> struct Pick<OP_ERODE> {
    static __device__ __forceinline__ uint32_t pick(uint32_t a, uint32_t b) { return a < b ? a : b; }
    static __device__ __forceinline__ float pick(float a, float b) { return __builtin_fminf(a, b); }
    static __device__ __forceinline__ double pick(double a, double b) { return __builtin_fmin(a, b); }
    static __device__ __forceinline__ uint32_t clamp(uint32_t a, uint32_t b) { return a > b ? a : b; }
    static __device__ __forceinline__ float clamp(float a, float b) { return __builtin_fmaxf(a, b); }
    static __device__ __forceinline__ double clamp(double a, double b) { return __builtin_fmax(a, b); }
};

// Cross-lane neighbours through DPP wave shifts.  from_left: lane i receives
// lane i-1 (the pixel to its left); from_right: lane i receives lane i+1.
// Lanes 0 / 63 receive 0: they sit on the region's outer edge, where wrong
// values are tolerated (see the header comment).
static constexpr int DPP_WAVE_SHR1 = 0x138;
static constexpr int DPP_WAVE_SHL1 = 0x130;

template <int CTRL>
__device__ __forceinline__ uint32_t lane_shift(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, true);
}
template <int CTRL>
__device__ __forceinline__ float lane_shift(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double lane_shift(double v) {
    uint64_t u = __builtin_bit_cast(uint64_t, v);
    uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, 0xF, 0xF, true);
    uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, true);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Two adjacent elements moved as one access (CW == 2 rows).
template <typename T> struct Pair;
template <> struct Pair<uint8_t> { using type = uint16_t; };
template <> struct Pair<float> { using type = float2; };
template <> struct Pair<double> { using type = double2; };

__device__ __forceinline__ void split_pair(uint16_t p, uint32_t &a, uint32_t &b) { a = p & 0xFFu; b = p >> 8; }
__device__ __forceinline__ void split_pair(float2 p, float &a, float &b) { a = p.x; b = p.y; }
__device__ __forceinline__ void split_pair(double2 p, double &a, double &b) { a = p.x; b = p.y; }
__device__ __forceinline__ uint16_t make_pair(uint32_t a, uint32_t b, uint8_t *) { return (uint16_t)(a | (b << 8)); }
__device__ __forceinline__ float2 make_pair(float a, float b, float *) { return make_float2(a, b); }
__device__ __forceinline__ double2 make_pair(double a, double b, double *) { return make_double2(a, b); }

template <typename T>
__device__ __forceinline__ bool pair_aligned(const T *p) {
    return ((uintptr_t)p & (2 * sizeof(T) - 1)) == 0;
}

__device__ __forceinline__ uint32_t to_reg(uint8_t v) { return v; }
__device__ __forceinline__ float to_reg(float v) { return v; }
__device__ __forceinline__ double to_reg(double v) { return v; }
__device__ __forceinline__ void from_reg(uint8_t *p, uint32_t v) { *p = (uint8_t)v; }
__device__ __forceinline__ void from_reg(float *p, float v) { *p = v; }
__device__ __forceinline__ void from_reg(double *p, double v) { *p = v; }

struct BlockArgs {
    const void *src;       // state before the block (marker for the first)
    const void *mask;      // mask image (geodesic mode), else unused
    void *dst;             // state after the block (core pixels written)
    int32_t width, height; // X, Y
    int64_t pitch;         // elements
    int32_t k;             // steps in this launch, 1 <= k <= halo
    int32_t halo;          // offset of the core inside the region
    int32_t core_x, core_y;
    int32_t tiles_x;
    int32_t tile0;         // tile of the launch's first workgroup (large images take several launches)
    int32_t tiles_per_image;   // batches of equal images: tiles of one image (0: a single image)
    int64_t image_stride;      // batches: elements between images of src, mask and dst
    uint32_t *change_word;       // reconstruction: OR of per-step change bits
    const uint32_t *prev_word;   // reconstruction: predecessor's word (or null)
    uint32_t prev_full;          // value prev_word holds if every step changed
    uint64_t erode_bits;         // MODE_MIXED: bit s set = step s of the launch erodes
};

// One workgroup = one tile.  CLAMP=false is the plain-chain body for regions
// that lie entirely inside the image (nothing to fence).
// Runs a.k steps on the region whose top-left corner is (rx0, ry0) and
// writes its core (offset a.halo, size core_x x core_y).  With DETECT, returns
// this wave's change bits (bit s: some core pixel changed at step s).
// A lane's CW adjacent exchange values in one LDS access where they span 8
// or 16 bytes (the exchange rows are 16-byte aligned): one 64-bit read
// instead of two interleaved 32-bit ones, which would meet two-way bank
// conflicts.
template <int CW, typename R>
__device__ __forceinline__ void read_cols(const R *p, R (&out)[CW]) {
    constexpr int B = CW * (int)sizeof(R);
    if constexpr (B == 8) {
        const uint2 v = *reinterpret_cast<const uint2 *>(p);
        __builtin_memcpy(out, &v, B);
    } else if constexpr (B == 16) {
        const uint4 v = *reinterpret_cast<const uint4 *>(p);
        __builtin_memcpy(out, &v, B);
    } else {
#pragma unroll
        for (int c = 0; c < CW; ++c) out[c] = p[c];
    }
}

// Core stores coherent at agent scope on their own (relaxed agent-scope
// atomic stores), for kernels that publish tiles to other workgroups: the
// release that follows then has (almost) nothing left to write back.
template <typename U>
__device__ __forceinline__ void agent_store(U *p, U v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void agent_store_pair(uint8_t *p, uint32_t a, uint32_t b) {
    agent_store(reinterpret_cast<uint16_t *>(p), (uint16_t)(a | (b << 8)));
}
__device__ __forceinline__ void agent_store_pair(float *p, float a, float b) {
    agent_store(reinterpret_cast<uint64_t *>(p),
                (uint64_t)__builtin_bit_cast(uint32_t, a) | ((uint64_t)__builtin_bit_cast(uint32_t, b) << 32));
}
__device__ __forceinline__ void agent_store_pair(double *p, double a, double b) {
    agent_store(p, a);
    agent_store(p + 1, b);
}
__device__ __forceinline__ void agent_store_reg(uint8_t *p, uint32_t v) { agent_store(p, (uint8_t)v); }
__device__ __forceinline__ void agent_store_reg(float *p, float v) { agent_store(p, v); }
__device__ __forceinline__ void agent_store_reg(double *p, double v) { agent_store(p, v); }

// Mixed chains hold the dilation fence of a plain chain (top inside the
// image, bottom outside); the erosion fence swaps the two values.
__device__ __forceinline__ uint32_t erosion_fence(uint32_t m) { return 255u - m; }
__device__ __forceinline__ float erosion_fence(float m) { return -m; }
__device__ __forceinline__ double erosion_fence(double m) { return -m; }

template <typename T, int OP, int MODE, bool CLAMP, bool DETECT, int CW, int RPW, int NW, bool AGENT_STORES = false>
__device__ __forceinline__ uint32_t chain_block_body(const BlockArgs &a, int rx0, int ry0,
                                                     typename RegOf<T>::type (*xch)[NW][2][64 * CW]) {
    using R = typename RegOf<T>::type;
    using B = Bounds<R, OP>;
    using P = Pick<OP>;
    static_assert(MODE != MODE_MIXED || OP == OP_DILATE, "mixed chains hold the dilation form of the fence");
    // State outside the image starts at the neutral value of the first
    // step's op (for mixed chains a run-time choice).
    R sbot = B::bottom();
    if constexpr (MODE == MODE_MIXED) sbot = (a.erode_bits & 1) ? Bounds<R, OP_ERODE>::bottom() : B::bottom();

    const int lane = threadIdx.x & 63;
    // wave index, known uniform: keeps the exchange branches scalar
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const T *src = static_cast<const T *>(a.src);
    const T *msk = static_cast<const T *>(a.mask);
    T *dst = static_cast<T *>(a.dst);
    const int k = a.k;
    const int halo = a.halo;

    R v[RPW][CW];
    R m[CLAMP ? RPW : 1][CLAMP ? CW : 1];

    // ---- load region (state and mask) ----
    // Fast path (uniform per workgroup): the region lies inside the image and
    // every lane's column pair is aligned, so each row is one access per lane
    // and array with no bounds checks and no divergent branches.
    constexpr int RX = 64 * CW;
    constexpr int RY = NW * RPW;
    bool fast = false;
    if constexpr (CW == 2) {
        fast = rx0 >= 0 && ry0 >= 0 && rx0 + RX <= a.width && ry0 + RY <= a.height && (rx0 & 1) == 0 &&
               (a.pitch & 1) == 0 && pair_aligned(src) && (MODE != MODE_GEODESIC || pair_aligned(msk));
    }
    if (fast) {
        if constexpr (CW == 2) {
            using PT = typename Pair<T>::type;
            const int64_t base = (int64_t)(ry0 + w * RPW) * a.pitch + rx0 + lane * 2;
#pragma unroll
            for (int r = 0; r < RPW; ++r)
                split_pair(*reinterpret_cast<const PT *>(src + base + r * a.pitch), v[r][0], v[r][1]);
            if constexpr (CLAMP) {
#pragma unroll
                for (int r = 0; r < RPW; ++r) {
                    if constexpr (MODE == MODE_GEODESIC)
                        split_pair(*reinterpret_cast<const PT *>(msk + base + r * a.pitch), m[r][0], m[r][1]);
                    else
                        m[r][0] = m[r][1] = B::top();
                }
            }
        }
    } else {
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
            const int y = ry0 + w * RPW + r;
            const bool yin = (unsigned)y < (unsigned)a.height;
#pragma unroll
            for (int c = 0; c < CW; ++c) {
                const int x = rx0 + lane * CW + c;
                const bool in = yin && (unsigned)x < (unsigned)a.width;
                const int64_t off = (int64_t)y * a.pitch + x;
                v[r][c] = in ? to_reg(src[off]) : sbot;
                if constexpr (CLAMP) {
                    if constexpr (MODE == MODE_GEODESIC)
                        m[r][c] = in ? to_reg(msk[off]) : B::bottom();
                    else
                        m[r][c] = in ? B::top() : B::bottom();
                }
            }
        }
    }

    // Column ownership of the core, for change detection.
    uint64_t col_in_core[CW];
    if constexpr (DETECT) {
#pragma unroll
        for (int c = 0; c < CW; ++c) {
            const int cx = lane * CW + c;
            const int x = rx0 + cx;
            const bool ok = cx >= halo && cx < halo + a.core_x && x < a.width;
            col_in_core[c] = __builtin_amdgcn_ballot_w64(ok);
        }
    }
    uint32_t step_bits = 0;

    // Rows still needed after step s: within k-1-s of the core, plus one row
    // either side for the row pass.  That band only shrinks, so each wave is
    // busy up to some step and idle from then on; an idle wave only takes
    // the barriers (its stale rows are never read by a needed row again).
    // Splitting the loop there keeps each step one branch-free block, which
    // lets the compiler overlap the LDS exchange with the column pass.
    const int busy_a = w * RPW + RPW - (halo - k);            // s < busy_a
    const int busy_b = halo + a.core_y + k - w * RPW;          // s < busy_b
    const int busy = __builtin_amdgcn_readfirstlane(max(0, min(k, min(busy_a, busy_b))));

    // Only waves holding core rows track changes; the others run the same
    // steps without the comparisons (one loop per case, each branch-free).
    //
    // The steps are software-pipelined across the barrier: after the column
    // pass of step s, a wave first computes the row pass of its two edge rows
    // for step s+1, publishes them (LDS write, barrier, LDS reads of the
    // neighbours' edges) and only then does the row pass of its middle rows
    // and, in the next iteration, their column pass -- work that needs no
    // LDS data and so covers the latency of the reads.  Every wave still
    // takes exactly k barriers.
    const bool wave_has_core = DETECT && w * RPW + RPW > halo && w * RPW < halo + a.core_y;
    auto run_steps = [&](auto detect_tag) {
        constexpr bool D = decltype(detect_tag)::value;
        if (busy == 0) return;
        R h[RPW][CW];
        R above[CW], below[CW];
        const int wa = w > 0 ? w - 1 : NW - 1;   // the first / last wave reads its own
        const int wb = w < NW - 1 ? w + 1 : 0;   // opposite edge: wrong, but on the region's edge
        // ---- row pass of one row (Section 3.1) ----
        auto row_pass = [&](int r) {
            const R left = lane_shift<DPP_WAVE_SHR1>(v[r][CW - 1]);
            const R right = lane_shift<DPP_WAVE_SHL1>(v[r][0]);
            if constexpr (CW == 1) {
                h[r][0] = P::pick(P::pick(left, v[r][0]), right);
            } else if constexpr (CW == 2) {
                // The pair's own extremum is shared by both outputs; each
                // output then takes one cross-lane neighbour, which the
                // compiler folds into a single DPP-sourced max/min.
                const R t = P::pick(v[r][0], v[r][1]);
                h[r][0] = P::pick(t, left);
                h[r][1] = P::pick(t, right);
            } else {
#pragma unroll
                for (int c = 0; c < CW; ++c) {
                    const R l = c == 0 ? left : v[r][c - 1];
                    const R rr = c == CW - 1 ? right : v[r][c + 1];
                    h[r][c] = P::pick(P::pick(v[r][c], rr), l);
                }
            }
        };
        // ---- edge rows to the waves above and below, through LDS ----
        auto publish = [&](int par) {
#pragma unroll
            for (int c = 0; c < CW; ++c) {
                xch[par][w][0][lane * CW + c] = h[0][c];
                xch[par][w][1][lane * CW + c] = h[RPW - 1][c];
            }
            __syncthreads();
            read_cols<CW>(&xch[par][wa][1][lane * CW], above);
            read_cols<CW>(&xch[par][wb][0][lane * CW], below);
        };
        // ---- column pass + clamp of one row ----
        auto column_pass = [&](int r, R (&nv)[RPW][CW], uint64_t &changed) {
            const int ry = w * RPW + r;
            const bool row_in_core = D && ry >= halo && ry < halo + a.core_y && ry0 + ry < a.height;
#pragma unroll
            for (int c = 0; c < CW; ++c) {
                const R up = r == 0 ? above[c] : h[r - 1][c];
                const R dn = r == RPW - 1 ? below[c] : h[r + 1][c];
                R x = P::pick(P::pick(up, h[r][c]), dn);
                if constexpr (CLAMP) x = P::clamp(x, m[r][c]);
                if constexpr (D) {
                    // branch-free: a uniform row mask instead of an if
                    const uint64_t row_mask = row_in_core ? ~0ull : 0ull;
                    changed |= __builtin_amdgcn_ballot_w64(x != v[r][c]) & col_in_core[c] & row_mask;
                }
                nv[r][c] = x;
            }
        };

        if constexpr (MODE == MODE_MIXED) {
            // Each step takes the extremum of its own op (bit s of
            // erode_bits: erosion); after a step the border fence pins
            // outside pixels to the neutral value of the op that reads the
            // state next.  Four copies of the step body, chosen by a uniform
            // branch on the ops of this step and the next.
            const uint64_t eb = a.erode_bits;
            auto row_pass_op = [&](auto op_tag, int r) {
                using PO = Pick<decltype(op_tag)::value>;
                const R left = lane_shift<DPP_WAVE_SHR1>(v[r][CW - 1]);
                const R right = lane_shift<DPP_WAVE_SHL1>(v[r][0]);
                if constexpr (CW == 1) {
                    h[r][0] = PO::pick(PO::pick(left, v[r][0]), right);
                } else if constexpr (CW == 2) {
                    const R t = PO::pick(v[r][0], v[r][1]);
                    h[r][0] = PO::pick(t, left);
                    h[r][1] = PO::pick(t, right);
                } else {
#pragma unroll
                    for (int c = 0; c < CW; ++c) {
                        const R l = c == 0 ? left : v[r][c - 1];
                        const R rr = c == CW - 1 ? right : v[r][c + 1];
                        h[r][c] = PO::pick(PO::pick(v[r][c], rr), l);
                    }
                }
            };
            auto step_op = [&](int s, auto cur_tag, auto next_tag) {
                using PC = Pick<decltype(cur_tag)::value>;
                R nv[RPW][CW];
                auto col = [&](int r) {
#pragma unroll
                    for (int c = 0; c < CW; ++c) {
                        const R up = r == 0 ? above[c] : h[r - 1][c];
                        const R dn = r == RPW - 1 ? below[c] : h[r + 1][c];
                        R x = PC::pick(PC::pick(up, h[r][c]), dn);
                        if constexpr (CLAMP) {
                            if constexpr (decltype(next_tag)::value == OP_DILATE)
                                x = Pick<OP_DILATE>::clamp(x, m[r][c]);
                            else
                                x = Pick<OP_ERODE>::clamp(x, erosion_fence(m[r][c]));
                        }
                        nv[r][c] = x;
                    }
                };
#pragma unroll
                for (int r = 1; r < RPW - 1; ++r) col(r);
                __builtin_amdgcn_sched_barrier(0);
                col(0);
                if constexpr (RPW > 1) col(RPW - 1);
#pragma unroll
                for (int r = 0; r < RPW; ++r)
#pragma unroll
                    for (int c = 0; c < CW; ++c) v[r][c] = nv[r][c];
                if (s + 1 < busy) {
                    row_pass_op(next_tag, 0);
                    if constexpr (RPW > 1) row_pass_op(next_tag, RPW - 1);
                    publish((s + 1) & 1);
#pragma unroll
                    for (int r = 1; r < RPW - 1; ++r) row_pass_op(next_tag, r);
                }
            };
            using DIL = std::integral_constant<int, OP_DILATE>;
            using ERO = std::integral_constant<int, OP_ERODE>;
            if (eb & 1) {
#pragma unroll
                for (int r = 0; r < RPW; ++r) row_pass_op(ERO{}, r);
            } else {
#pragma unroll
                for (int r = 0; r < RPW; ++r) row_pass_op(DIL{}, r);
            }
            publish(0);
            for (int s = 0; s < busy; ++s) {
                const bool ce = (eb >> s) & 1;
                const bool ne = s + 1 < k ? ((eb >> (s + 1)) & 1) : ce;
                if (ce) {
                    if (ne) step_op(s, ERO{}, ERO{});
                    else step_op(s, ERO{}, DIL{});
                } else {
                    if (ne) step_op(s, DIL{}, ERO{});
                    else step_op(s, DIL{}, DIL{});
                }
            }
            return;
        }

#pragma unroll
        for (int r = 0; r < RPW; ++r) row_pass(r);
        publish(0);
        // (64-bit registers keep the one-step loop: the second state array
        // costs them more in register pressure than the copies)
        if constexpr (!D || sizeof(R) > 4) {
            for (int s = 0; s < busy; ++s) {
                R nv[RPW][CW];
                uint64_t changed = 0;
#pragma unroll
                for (int r = 1; r < RPW - 1; ++r) column_pass(r, nv, changed);
                // the edge rows, which wait for the exchange reads, after the
                // middle rows, which cover the reads' latency
                __builtin_amdgcn_sched_barrier(0);
                column_pass(0, nv, changed);
                if constexpr (RPW > 1) column_pass(RPW - 1, nv, changed);
#pragma unroll
                for (int r = 0; r < RPW; ++r)
#pragma unroll
                    for (int c = 0; c < CW; ++c) v[r][c] = nv[r][c];
                if constexpr (D) {
                    if (changed) step_bits |= 1u << s;
                }
                if (s + 1 < busy) {
                    row_pass(0);
                    if constexpr (RPW > 1) row_pass(RPW - 1);
                    publish((s + 1) & 1);
#pragma unroll
                    for (int r = 1; r < RPW - 1; ++r) row_pass(r);
                }
            }
        } else {
            // As in the packed body: two steps per iteration with the old and
            // new states in alternating arrays, so the change test's reads of
            // the old state need no register copies.
            R v2[RPW][CW];
            auto row_pass_of = [&](R (&st)[RPW][CW], int r) {
                const R left = lane_shift<DPP_WAVE_SHR1>(st[r][CW - 1]);
                const R right = lane_shift<DPP_WAVE_SHL1>(st[r][0]);
                if constexpr (CW == 1) {
                    h[r][0] = P::pick(P::pick(left, st[r][0]), right);
                } else if constexpr (CW == 2) {
                    const R t = P::pick(st[r][0], st[r][1]);
                    h[r][0] = P::pick(t, left);
                    h[r][1] = P::pick(t, right);
                } else {
#pragma unroll
                    for (int c = 0; c < CW; ++c) {
                        const R l = c == 0 ? left : st[r][c - 1];
                        const R rr = c == CW - 1 ? right : st[r][c + 1];
                        h[r][c] = P::pick(P::pick(st[r][c], rr), l);
                    }
                }
            };
            auto step = [&](int s, R (&cur)[RPW][CW], R (&nxt)[RPW][CW]) {
                uint64_t changed = 0;
                auto col = [&](int r) {
                    const int ry = w * RPW + r;
                    const bool row_in_core = ry >= halo && ry < halo + a.core_y && ry0 + ry < a.height;
#pragma unroll
                    for (int c = 0; c < CW; ++c) {
                        const R up = r == 0 ? above[c] : h[r - 1][c];
                        const R dn = r == RPW - 1 ? below[c] : h[r + 1][c];
                        R x = P::pick(P::pick(up, h[r][c]), dn);
                        if constexpr (CLAMP) x = P::clamp(x, m[r][c]);
                        const uint64_t row_mask = row_in_core ? ~0ull : 0ull;
                        changed |= __builtin_amdgcn_ballot_w64(x != cur[r][c]) & col_in_core[c] & row_mask;
                        nxt[r][c] = x;
                    }
                };
#pragma unroll
                for (int r = 1; r < RPW - 1; ++r) col(r);
                __builtin_amdgcn_sched_barrier(0);
                col(0);
                if constexpr (RPW > 1) col(RPW - 1);
                if (changed) step_bits |= 1u << s;
                if (s + 1 < busy) {
                    row_pass_of(nxt, 0);
                    if constexpr (RPW > 1) row_pass_of(nxt, RPW - 1);
                    publish((s + 1) & 1);
#pragma unroll
                    for (int r = 1; r < RPW - 1; ++r) row_pass_of(nxt, r);
                }
            };
            int s = 0;
            for (; s + 1 < busy; s += 2) {
                step(s, v, v2);
                step(s + 1, v2, v);
            }
            if (s < busy) {
                step(s, v, v2);
#pragma unroll
                for (int r = 0; r < RPW; ++r)
#pragma unroll
                    for (int c = 0; c < CW; ++c) v[r][c] = v2[r][c];
            }
        }
    };
    if (wave_has_core)
        run_steps(std::true_type{});
    else
        run_steps(std::false_type{});
    for (int s = busy; s < k; ++s) __syncthreads();

    // ---- store the core ----
    // Pairs whose two columns are both core pixels inside the image go out as
    // one access when aligned (all of them on the fast path); the rest one by
    // one.  Stores need no waits, so the per-lane conditions cost little.
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
        const int ry = w * RPW + r;
        const int y = ry0 + ry;
        const bool yok = ry >= halo && ry < halo + a.core_y && y < a.height;
        if (!yok) continue;
        if constexpr (CW == 2) {
            const int cx = lane * 2;
            const int x = rx0 + cx;
            T *p = dst + (int64_t)y * a.pitch + x;
            const bool in0 = cx >= halo && cx < halo + a.core_x && x < a.width;
            const bool in1 = cx + 1 >= halo && cx + 1 < halo + a.core_x && x + 1 < a.width;
            if (in0 && in1 && (fast || pair_aligned(p))) {
                if constexpr (AGENT_STORES) {
                    agent_store_pair(p, v[r][0], v[r][1]);
                } else {
                    using PT = typename Pair<T>::type;
                    *reinterpret_cast<PT *>(p) = make_pair(v[r][0], v[r][1], p);
                }
            } else if constexpr (AGENT_STORES) {
                if (in0) agent_store_reg(p, v[r][0]);
                if (in1) agent_store_reg(p + 1, v[r][1]);
            } else {
                if (in0) from_reg(p, v[r][0]);
                if (in1) from_reg(p + 1, v[r][1]);
            }
        } else {
#pragma unroll
            for (int c = 0; c < CW; ++c) {
                const int cx = lane * CW + c;
                const int x = rx0 + cx;
                if (cx >= halo && cx < halo + a.core_x && x < a.width) {
                    if constexpr (AGENT_STORES)
                        agent_store_reg(dst + (int64_t)y * a.pitch + x, v[r][c]);
                    else
                        from_reg(dst + (int64_t)y * a.pitch + x, v[r][c]);
                }
            }
        }
    }
    return step_bits;
}

// Two-group layout: a wave covers RX = 32*CW columns and 2*RPW rows.
// Lanes 0..31 (group 0) hold the wave's first RPW rows, lanes 32..63 (group
// 1) the next RPW rows; lane l holds columns [(l%32)*CW, (l%32+1)*CW).  The
// DPP wave shifts of the row pass cross from lane 31 to lane 32 only at the
// region's left/right edge, where wrong values are tolerated.  Every group
// publishes its first and last row-pass rows in LDS and reads the row above
// and below it from there (per-lane addresses, no selects).  A narrower
// region (96 columns for CW = 3) lets a 64 x 64 core run with a 16-pixel
// halo instead of 32.
template <typename T, int OP, int MODE, bool CLAMP, bool DETECT, int CW, int RPW, int NW>
__device__ __forceinline__ uint32_t chain_block_body_g2(const BlockArgs &a, int rx0, int ry0,
                                                        typename RegOf<T>::type (*xch)[NW][4][32 * CW]) {
    using R = typename RegOf<T>::type;
    using B = Bounds<R, OP>;
    using P = Pick<OP>;
    constexpr int RX = 32 * CW;
    constexpr int WR = 2 * RPW;  // rows per wave
    constexpr int RY = NW * WR;

    const int lane = threadIdx.x & 63;
    const int grp = lane >> 5;
    const int lc = lane & 31;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int row0 = w * WR + grp * RPW;  // first region row of this lane
    const T *src = static_cast<const T *>(a.src);
    const T *msk = static_cast<const T *>(a.mask);
    T *dst = static_cast<T *>(a.dst);
    const int k = a.k;
    const int halo = a.halo;

    R v[RPW][CW];
    R m[CLAMP ? RPW : 1][CLAMP ? CW : 1];

    // ---- load region ----
    const bool inside = rx0 >= 0 && ry0 >= 0 && rx0 + RX <= a.width && ry0 + RY <= a.height;
    if (inside) {
        const int64_t base = (int64_t)(ry0 + row0) * a.pitch + rx0 + lc * CW;
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
#pragma unroll
            for (int c = 0; c < CW; ++c) {
                v[r][c] = to_reg(src[base + r * a.pitch + c]);
                if constexpr (CLAMP) {
                    if constexpr (MODE == MODE_GEODESIC)
                        m[r][c] = to_reg(msk[base + r * a.pitch + c]);
                    else
                        m[r][c] = B::top();
                }
            }
        }
    } else {
#pragma unroll
        for (int r = 0; r < RPW; ++r) {
            const int y = ry0 + row0 + r;
            const bool yin = (unsigned)y < (unsigned)a.height;
#pragma unroll
            for (int c = 0; c < CW; ++c) {
                const int x = rx0 + lc * CW + c;
                const bool in = yin && (unsigned)x < (unsigned)a.width;
                const int64_t off = (int64_t)y * a.pitch + x;
                v[r][c] = in ? to_reg(src[off]) : B::bottom();
                if constexpr (CLAMP) {
                    if constexpr (MODE == MODE_GEODESIC)
                        m[r][c] = in ? to_reg(msk[off]) : B::bottom();
                    else
                        m[r][c] = in ? B::top() : B::bottom();
                }
            }
        }
    }

    // Core ownership for change detection (per lane: rows depend on group).
    uint64_t col_in_core[CW];
    if constexpr (DETECT) {
#pragma unroll
        for (int c = 0; c < CW; ++c) {
            const int cx = lc * CW + c;
            col_in_core[c] = __builtin_amdgcn_ballot_w64(cx >= halo && cx < halo + a.core_x &&
                                                         rx0 + cx < a.width);
        }
    }
    uint32_t step_bits = 0;

    // Idle from the step on which the wave's rows leave the needed band (see
    // chain_block_body).
    const int busy_a = w * WR + WR - (halo - k);
    const int busy_b = halo + a.core_y + k - w * WR;
    const int busy = __builtin_amdgcn_readfirstlane(max(0, min(k, min(busy_a, busy_b))));
    // LDS slots per wave: [group * 2 + 0] first row, [group * 2 + 1] last
    // row.  The row above a group's first row is the last row of the group
    // before it (group 1 of the wave above for group 0); the row below its
    // last row is the first row of the group after it (wrapping at the
    // region's edge: harmless there).
    const int wa = w > 0 ? w - 1 : NW - 1;
    const int wb = w < NW - 1 ? w + 1 : 0;
    const int above_w = grp ? w : wa, above_slot = grp ? 1 : 3;
    const int below_w = grp ? wb : w, below_slot = grp ? 0 : 2;

    const bool wave_has_core = DETECT && w * WR + WR > halo && w * WR < halo + a.core_y;
    auto run_steps = [&](auto detect_tag) {
        constexpr bool D = decltype(detect_tag)::value;
        for (int s = 0; s < busy; ++s) {
            // ---- 1. row pass ----
            R h[RPW][CW];
#pragma unroll
            for (int r = 0; r < RPW; ++r) {
                const R left = lane_shift<DPP_WAVE_SHR1>(v[r][CW - 1]);
                const R right = lane_shift<DPP_WAVE_SHL1>(v[r][0]);
                if constexpr (CW == 3) {
                    // Both partial extrema feed two outputs each, so the
                    // compiler keeps them and folds the neighbour lanes into
                    // DPP-sourced max/min: 5 operations for 3 pixels.
                    const R t1 = P::pick(v[r][0], v[r][1]);
                    const R t2 = P::pick(v[r][1], v[r][2]);
                    h[r][0] = P::pick(t1, left);
                    h[r][1] = P::pick(t1, t2);
                    h[r][2] = P::pick(t2, right);
                } else {
#pragma unroll
                    for (int c = 0; c < CW; ++c) {
                        const R l = c == 0 ? left : v[r][c - 1];
                        const R rr = c == CW - 1 ? right : v[r][c + 1];
                        h[r][c] = P::pick(P::pick(v[r][c], rr), l);
                    }
                }
            }
            // ---- 2. exchange through LDS ----
            const int par = s & 1;
#pragma unroll
            for (int c = 0; c < CW; ++c) {
                xch[par][w][grp * 2][lc * CW + c] = h[0][c];
                xch[par][w][grp * 2 + 1][lc * CW + c] = h[RPW - 1][c];
            }
            __syncthreads();
            R above[CW], below[CW];
#pragma unroll
            for (int c = 0; c < CW; ++c) {
                above[c] = xch[par][above_w][above_slot][lc * CW + c];
                below[c] = xch[par][below_w][below_slot][lc * CW + c];
            }
            // ---- 3. column pass + clamp ----
            uint64_t changed = 0;
#pragma unroll
            for (int r = 0; r < RPW; ++r) {
                const int ry = row0 + r;
                const bool row_in_core = D && ry >= halo && ry < halo + a.core_y && ry0 + ry < a.height;
#pragma unroll
                for (int c = 0; c < CW; ++c) {
                    const R up = r == 0 ? above[c] : h[r - 1][c];
                    const R dn = r == RPW - 1 ? below[c] : h[r + 1][c];
                    R nv = P::pick(P::pick(up, h[r][c]), dn);
                    if constexpr (CLAMP) nv = P::clamp(nv, m[r][c]);
                    if constexpr (D)
                        changed |= __builtin_amdgcn_ballot_w64(row_in_core && nv != v[r][c]) & col_in_core[c];
                    v[r][c] = nv;
                }
            }
            if constexpr (D) {
                if (changed) step_bits |= 1u << s;
            }
        }
    };
    if (wave_has_core)
        run_steps(std::true_type{});
    else
        run_steps(std::false_type{});
    for (int s = busy; s < k; ++s) __syncthreads();

    // ---- store the core ----
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
        const int ry = row0 + r;
        const int y = ry0 + ry;
        if (!(ry >= halo && ry < halo + a.core_y && y < a.height)) continue;
#pragma unroll
        for (int c = 0; c < CW; ++c) {
            const int cx = lc * CW + c;
            const int x = rx0 + cx;
            if (cx >= halo && cx < halo + a.core_x && x < a.width)
                from_reg(dst + (int64_t)y * a.pitch + x, v[r][c]);
        }
    }
    return step_bits;
}

// ---------------------------------------------------------------------------
// u8 body with two rows per register.  Register row j of a wave holds its
// region rows j (low 16 bits) and j + RPW/2 (high 16 bits), so each packed
// instruction handles two pixels; both rows belong to the same wave, so the
// busy band, the edge exchange and the row pass are those of
// chain_block_body.  The column pass meets the halves' seams twice: the row
// above register 0's low half is the wave above's last row (the high half of
// its last register) and the row above its high half is this wave's
// register RPW/2 - 1, low half; one funnel shift (alignbit) builds each seam
// operand, and likewise below the last register.
//
// A pixel value p in 0..255 is held as the half-precision number 1024 + p,
// whose bit pattern is 0x6400 | p (binary16 has unit spacing on
// [1024, 2048)).  Encoding and decoding are a bit-or and taking the low
// byte, the encoding preserves order, and the packed three-input
// half-precision maximum/minimum then takes the extremum of three pixel
// pairs in one instruction, exactly.  No NaN, infinity or -0 can arise.
// ---------------------------------------------------------------------------
typedef _Float16 gc_f16x2 __attribute__((ext_vector_type(2)));

constexpr uint32_t PK_BIAS = 0x64006400u;  // 1024 in both halves

template <int OP> struct PackedPick;
template <> struct PackedPick<OP_DILATE> {
    static __device__ __forceinline__ gc_f16x2 hx(uint32_t a) { return __builtin_bit_cast(gc_f16x2, a); }
    static __device__ __forceinline__ uint32_t pick(uint32_t a, uint32_t b) {
        return __builtin_bit_cast(uint32_t, __builtin_elementwise_maximum(hx(a), hx(b)));
    }
    static __device__ __forceinline__ uint32_t pick3(uint32_t a, uint32_t b, uint32_t c) {
        return __builtin_bit_cast(uint32_t,
                                  __builtin_elementwise_maximum(__builtin_elementwise_maximum(hx(a), hx(b)), hx(c)));
    }
    static __device__ __forceinline__ uint32_t clamp(uint32_t a, uint32_t b) {
        return __builtin_bit_cast(uint32_t, __builtin_elementwise_minimum(hx(a), hx(b)));
    }
};
template <> struct PackedPick<OP_ERODE> {
    static __device__ __forceinline__ gc_f16x2 hx(uint32_t a) { return __builtin_bit_cast(gc_f16x2, a); }
    static __device__ __forceinline__ uint32_t pick(uint32_t a, uint32_t b) {
        return PackedPick<OP_DILATE>::clamp(a, b);
    }
    static __device__ __forceinline__ uint32_t pick3(uint32_t a, uint32_t b, uint32_t c) {
        return __builtin_bit_cast(uint32_t,
                                  __builtin_elementwise_minimum(__builtin_elementwise_minimum(hx(a), hx(b)), hx(c)));
    }
    static __device__ __forceinline__ uint32_t clamp(uint32_t a, uint32_t b) {
        return PackedPick<OP_DILATE>::pick(a, b);
    }
};

// Two u8 values (0..255) -> one register of encoded halves.
__device__ __forceinline__ uint32_t pack_rows(uint32_t lo, uint32_t hi) { return lo | (hi << 16) | PK_BIAS; }

// Lanes per column group: 64 (one group) or 32 (two groups).
template <int OP, int MODE, bool CLAMP, bool DETECT, int RPW, int NW, bool AGENT_STORES = false,
          bool STAGED = false>
__device__ __forceinline__ uint32_t chain_block_body_pk(const BlockArgs &a, int rx0, int ry0,
                                                        uint32_t (*xch)[NW][2][128], uint8_t *stage) {
    static_assert(RPW % 2 == 0, "two rows per register");
    static_assert(MODE != MODE_MIXED || OP == OP_DILATE, "mixed chains hold the dilation form of the fence");
    constexpr int H = RPW / 2;      // registers per column
    constexpr int CW = 2;
    using B = Bounds<uint32_t, OP>;
    using P = PackedPick<OP>;
    // State outside the image starts at the neutral value of the first
    // step's op: for mixed chains a run-time choice (the fence keeps it
    // neutral for whichever op reads the state next).
    uint32_t sbot = B::bottom();
    if constexpr (MODE == MODE_MIXED) sbot = (a.erode_bits & 1) ? 255u : 0u;

    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint8_t *src = static_cast<const uint8_t *>(a.src);
    const uint8_t *msk = static_cast<const uint8_t *>(a.mask);
    uint8_t *dst = static_cast<uint8_t *>(a.dst);
    const int k = a.k;
    const int halo = a.halo;
    constexpr int RX = 64 * CW;
    constexpr int RY = NW * RPW;

    uint32_t v[H][CW];
    uint32_t m[CLAMP ? H : 1][CW];

    // ---- load region (rows j and j + H into register j) ----
    // STAGED (per-launch kernel): through LDS, see below; otherwise (the
    // persistent kernel, whose second workgroup per CU hides the loads) one
    // two-byte access per lane, row pair and image.
    // The store at the end follows the same choice.
    bool fast = false;
    if constexpr (STAGED) {
        // Staged through LDS: the workgroup reads the region in 16-byte chunks of
        // its rows, one wide load per chunk and image (at most two per thread),
        // then each lane picks its two columns of its rows out of LDS.  Chunks
        // outside the image are filled with the neutral value; a chunk that
        // straddles the image border, or is not 16-byte aligned, is read byte by
        // byte behind the inside-the-image test.
        {
            constexpr int CH = RX / 16;     // chunks per region row
            constexpr int NCH = RY * CH;    // chunks per image
            uint8_t *sv = stage;            // RY x RX state
            uint8_t *sm = stage + RY * RX;  // RY x RX mask (clamped bodies)
            const uint32_t bot4 = B::bottom() * 0x01010101u;
            const uint32_t sbot4 = sbot * 0x01010101u;
            const uint32_t top4 = B::top() * 0x01010101u;
            for (int i = threadIdx.x; i < NCH; i += 64 * NW) {
                const int r = i / CH, c = i % CH;
                const int y = ry0 + r, x = rx0 + 16 * c;
                const bool yin = (unsigned)y < (unsigned)a.height;
                const int64_t off = (int64_t)y * a.pitch + x;
                uint4 cv = make_uint4(sbot4, sbot4, sbot4, sbot4);
                uint4 cm = make_uint4(bot4, bot4, bot4, bot4);
                const bool whole = yin && x >= 0 && x + 16 <= a.width;
                const bool none = !yin || x + 16 <= 0 || x >= a.width;
                if (whole && ((uintptr_t)(src + off) & 15) == 0 &&
                    (MODE != MODE_GEODESIC || ((uintptr_t)(msk + off) & 15) == 0)) {
                    cv = *reinterpret_cast<const uint4 *>(src + off);
                    if constexpr (CLAMP) {
                        if constexpr (MODE == MODE_GEODESIC)
                            cm = *reinterpret_cast<const uint4 *>(msk + off);
                        else
                            cm = make_uint4(top4, top4, top4, top4);
                    }
                } else if (!none) {
                    uint32_t wv[4], wm[4];
    #pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        wv[q] = 0;
                        wm[q] = 0;
    #pragma unroll
                        for (int b = 0; b < 4; ++b) {
                            const int xb = x + 4 * q + b;
                            const bool in = yin && (unsigned)xb < (unsigned)a.width;
                            const uint32_t pv = in ? (uint32_t)src[off + 4 * q + b] : sbot;
                            uint32_t pm = B::bottom();
                            if constexpr (MODE == MODE_GEODESIC)
                                pm = in ? (uint32_t)msk[off + 4 * q + b] : B::bottom();
                            else
                                pm = in ? B::top() : B::bottom();
                            wv[q] |= pv << (8 * b);
                            wm[q] |= pm << (8 * b);
                        }
                    }
                    cv = make_uint4(wv[0], wv[1], wv[2], wv[3]);
                    cm = make_uint4(wm[0], wm[1], wm[2], wm[3]);
                }
                *reinterpret_cast<uint4 *>(sv + r * RX + 16 * c) = cv;
                if constexpr (CLAMP) *reinterpret_cast<uint4 *>(sm + r * RX + 16 * c) = cm;
            }
            __syncthreads();
            const int base = (w * RPW) * RX + lane * 2;
    #pragma unroll
            for (int j = 0; j < H; ++j) {
                const uint32_t lo = *reinterpret_cast<const uint16_t *>(sv + base + j * RX);
                const uint32_t hi = *reinterpret_cast<const uint16_t *>(sv + base + (j + H) * RX);
                v[j][0] = pack_rows(lo & 0xFFu, hi & 0xFFu);
                v[j][1] = pack_rows(lo >> 8, hi >> 8);
                if constexpr (CLAMP) {
                    const uint32_t mlo = *reinterpret_cast<const uint16_t *>(sm + base + j * RX);
                    const uint32_t mhi = *reinterpret_cast<const uint16_t *>(sm + base + (j + H) * RX);
                    m[j][0] = pack_rows(mlo & 0xFFu, mhi & 0xFFu);
                    m[j][1] = pack_rows(mlo >> 8, mhi >> 8);
                }
            }
        }
    } else {
        fast = rx0 >= 0 && ry0 >= 0 && rx0 + RX <= a.width && ry0 + RY <= a.height && (rx0 & 1) == 0 &&
                          (a.pitch & 1) == 0 && pair_aligned(src) && (MODE != MODE_GEODESIC || pair_aligned(msk));
        if (fast) {
            const int64_t base = (int64_t)(ry0 + w * RPW) * a.pitch + rx0 + lane * 2;
    #pragma unroll
            for (int j = 0; j < H; ++j) {
                const uint32_t lo = *reinterpret_cast<const uint16_t *>(src + base + j * a.pitch);
                const uint32_t hi = *reinterpret_cast<const uint16_t *>(src + base + (j + H) * a.pitch);
                v[j][0] = pack_rows(lo & 0xFFu, hi & 0xFFu);
                v[j][1] = pack_rows(lo >> 8, hi >> 8);
                if constexpr (CLAMP) {
                    if constexpr (MODE == MODE_GEODESIC) {
                        const uint32_t mlo = *reinterpret_cast<const uint16_t *>(msk + base + j * a.pitch);
                        const uint32_t mhi = *reinterpret_cast<const uint16_t *>(msk + base + (j + H) * a.pitch);
                        m[j][0] = pack_rows(mlo & 0xFFu, mhi & 0xFFu);
                        m[j][1] = pack_rows(mlo >> 8, mhi >> 8);
                    } else {
                        m[j][0] = m[j][1] = pack_rows(B::top(), B::top());
                    }
                }
            }
        } else {
    #pragma unroll
            for (int j = 0; j < H; ++j) {
    #pragma unroll
                for (int c = 0; c < CW; ++c) {
                    const int x = rx0 + lane * CW + c;
                    const bool xin = (unsigned)x < (unsigned)a.width;
                    uint32_t vv[2], mm[2];
    #pragma unroll
                    for (int half = 0; half < 2; ++half) {
                        const int y = ry0 + w * RPW + j + half * H;
                        const bool in = xin && (unsigned)y < (unsigned)a.height;
                        const int64_t off = (int64_t)y * a.pitch + x;
                        vv[half] = in ? (uint32_t)src[off] : sbot;
                        if constexpr (MODE == MODE_GEODESIC)
                            mm[half] = in ? (uint32_t)msk[off] : B::bottom();
                        else
                            mm[half] = in ? B::top() : B::bottom();
                    }
                    v[j][c] = pack_rows(vv[0], vv[1]);
                    if constexpr (CLAMP) m[j][c] = pack_rows(mm[0], mm[1]);
                }
            }
        }
    }
    // Change detection: per register, the bits of its core pixels (16-bit
    // halves of core rows, in columns of the core).  A step changed the core
    // iff some (new ^ old) & mask is nonzero; the encodings are unique, so
    // equal bits mean equal pixels.
    uint32_t cmask[DETECT ? H : 1][CW];
    if constexpr (DETECT) {
#pragma unroll
        for (int j = 0; j < H; ++j) {
            const int ry = w * RPW + j;
            const bool lo = ry >= halo && ry < halo + a.core_y && ry0 + ry < a.height;
            const bool hi = ry + H >= halo && ry + H < halo + a.core_y && ry0 + ry + H < a.height;
#pragma unroll
            for (int c = 0; c < CW; ++c) {
                const int cx = lane * CW + c;
                const bool col = cx >= halo && cx < halo + a.core_x && rx0 + cx < a.width;
                cmask[j][c] = col ? ((lo ? 0x0000FFFFu : 0u) | (hi ? 0xFFFF0000u : 0u)) : 0u;
            }
        }
    }
    uint32_t step_bits = 0;

    const int busy_a = w * RPW + RPW - (halo - k);
    const int busy_b = halo + a.core_y + k - w * RPW;
    const int busy = __builtin_amdgcn_readfirstlane(max(0, min(k, min(busy_a, busy_b))));
    const bool wave_has_core = DETECT && w * RPW + RPW > halo && w * RPW < halo + a.core_y;

    auto run_steps = [&](auto detect_tag) {
        constexpr bool D = decltype(detect_tag)::value;
        if (busy == 0) return;
        uint32_t h[H][CW];
        uint32_t above[CW], below[CW];
        const int wa = w > 0 ? w - 1 : NW - 1;
        const int wb = w < NW - 1 ? w + 1 : 0;
        auto row_pass = [&](int j) {
            const uint32_t left = lane_shift<DPP_WAVE_SHR1>(v[j][1]);
            const uint32_t right = lane_shift<DPP_WAVE_SHL1>(v[j][0]);
            h[j][0] = P::pick3(left, v[j][0], v[j][1]);
            h[j][1] = P::pick3(v[j][0], v[j][1], right);
        };
        auto publish = [&](int par) {
#pragma unroll
            for (int c = 0; c < CW; ++c) {
                xch[par][w][0][lane * CW + c] = h[0][c];
                xch[par][w][1][lane * CW + c] = h[H - 1][c];
            }
            __syncthreads();
            read_cols<CW>(&xch[par][wa][1][lane * CW], above);
            read_cols<CW>(&xch[par][wb][0][lane * CW], below);
        };
        auto finish = [&](int j, int c, uint32_t x, uint32_t (&nv)[H][CW], uint32_t &changed) {
            if constexpr (CLAMP) x = P::clamp(x, m[j][c]);
            if constexpr (D) changed |= (x ^ v[j][c]) & cmask[j][c];
            nv[j][c] = x;
        };

        if constexpr (MODE == MODE_MIXED) {
            // Each step takes the extremum of its own op (bit s of
            // erode_bits: erosion).  The border fence after a step pins
            // outside pixels to the neutral value of the op that reads the
            // state next: m holds the dilation fence (255 inside, 0
            // outside), the erosion fence is the same with each pixel's
            // bits flipped (0 inside, 255 outside).  Steps go through one
            // of four copies of the step body, chosen by a uniform branch
            // on the ops of this step and the next.
            const uint64_t eb = a.erode_bits;
            auto row_pass_op = [&](auto op_tag, int j) {
                using PO = PackedPick<decltype(op_tag)::value>;
                const uint32_t left = lane_shift<DPP_WAVE_SHR1>(v[j][1]);
                const uint32_t right = lane_shift<DPP_WAVE_SHL1>(v[j][0]);
                h[j][0] = PO::pick3(left, v[j][0], v[j][1]);
                h[j][1] = PO::pick3(v[j][0], v[j][1], right);
            };
            auto step_op = [&](int s, auto cur_tag, auto next_tag) {
                using PC = PackedPick<decltype(cur_tag)::value>;
                uint32_t nv[H][CW];
                auto fin = [&](int j, int c, uint32_t x) {
                    if constexpr (CLAMP) {
                        if constexpr (decltype(next_tag)::value == OP_DILATE)
                            x = PackedPick<OP_DILATE>::clamp(x, m[j][c]);
                        else
                            x = PackedPick<OP_ERODE>::clamp(x, m[j][c] ^ 0x00FF00FFu);
                    }
                    nv[j][c] = x;
                };
#pragma unroll
                for (int c = 0; c < CW; ++c) {
#pragma unroll
                    for (int j = 1; j < H - 1; ++j) fin(j, c, PC::pick3(h[j - 1][c], h[j][c], h[j + 1][c]));
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int c = 0; c < CW; ++c) {
                    const uint32_t up0 = __builtin_amdgcn_alignbit(h[H - 1][c], above[c], 16);
                    const uint32_t dnl = __builtin_amdgcn_alignbit(below[c], h[0][c], 16);
                    if constexpr (H == 1) {
                        fin(0, c, PC::pick3(up0, h[0][c], dnl));
                    } else {
                        fin(0, c, PC::pick3(up0, h[0][c], h[1][c]));
                        fin(H - 1, c, PC::pick3(h[H - 2][c], h[H - 1][c], dnl));
                    }
                }
#pragma unroll
                for (int j = 0; j < H; ++j)
#pragma unroll
                    for (int c = 0; c < CW; ++c) v[j][c] = nv[j][c];
                if (s + 1 < busy) {
                    row_pass_op(next_tag, 0);
                    if constexpr (H > 1) row_pass_op(next_tag, H - 1);
                    publish((s + 1) & 1);
#pragma unroll
                    for (int j = 1; j < H - 1; ++j) row_pass_op(next_tag, j);
                }
            };
            using DIL = std::integral_constant<int, OP_DILATE>;
            using ERO = std::integral_constant<int, OP_ERODE>;
            if (eb & 1) {
#pragma unroll
                for (int j = 0; j < H; ++j) row_pass_op(ERO{}, j);
            } else {
#pragma unroll
                for (int j = 0; j < H; ++j) row_pass_op(DIL{}, j);
            }
            publish(0);
            for (int s = 0; s < busy; ++s) {
                const bool ce = (eb >> s) & 1;
                const bool ne = s + 1 < k ? ((eb >> (s + 1)) & 1) : ce;
                if (ce) {
                    if (ne) step_op(s, ERO{}, ERO{});
                    else step_op(s, ERO{}, DIL{});
                } else {
                    if (ne) step_op(s, DIL{}, ERO{});
                    else step_op(s, DIL{}, DIL{});
                }
            }
            return;
        }

#pragma unroll
        for (int j = 0; j < H; ++j) row_pass(j);
        publish(0);
        if constexpr (!D) {
            for (int s = 0; s < busy; ++s) {
                uint32_t nv[H][CW];
                uint32_t changed = 0;
#pragma unroll
                for (int c = 0; c < CW; ++c) {
#pragma unroll
                    for (int j = 1; j < H - 1; ++j) finish(j, c, P::pick3(h[j - 1][c], h[j][c], h[j + 1][c]), nv, changed);
                }
                // keep the seams, which wait for the exchange reads, after the
                // middle registers, which cover the reads' latency
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int c = 0; c < CW; ++c) {
                    // seams: rows above register 0 are (wave above's last row,
                    // this wave's row H - 1); rows below register H - 1 are
                    // (this wave's row H, wave below's first row)
                    const uint32_t up0 = __builtin_amdgcn_alignbit(h[H - 1][c], above[c], 16);
                    const uint32_t dnl = __builtin_amdgcn_alignbit(below[c], h[0][c], 16);
                    if constexpr (H == 1) {
                        finish(0, c, P::pick3(up0, h[0][c], dnl), nv, changed);
                    } else {
                        finish(0, c, P::pick3(up0, h[0][c], h[1][c]), nv, changed);
                        finish(H - 1, c, P::pick3(h[H - 2][c], h[H - 1][c], dnl), nv, changed);
                    }
                }
#pragma unroll
                for (int j = 0; j < H; ++j)
#pragma unroll
                    for (int c = 0; c < CW; ++c) v[j][c] = nv[j][c];
                if constexpr (D) {
                    if (__builtin_amdgcn_ballot_w64(changed != 0)) step_bits |= 1u << s;
                }
                if (s + 1 < busy) {
                    row_pass(0);
                    if constexpr (H > 1) row_pass(H - 1);
                    publish((s + 1) & 1);
#pragma unroll
                    for (int j = 1; j < H - 1; ++j) row_pass(j);
                }
            }
        } else {
            // With change detection each step reads the previous state after
            // the new one exists, so a loop that copies new into old would
            // move every register each step; two steps per iteration with the
            // roles of v and v2 swapped keep both in place.
            uint32_t v2[H][CW];
            auto row_pass_of = [&](uint32_t (&st)[H][CW], int j) {
                const uint32_t left = lane_shift<DPP_WAVE_SHR1>(st[j][1]);
                const uint32_t right = lane_shift<DPP_WAVE_SHL1>(st[j][0]);
                h[j][0] = P::pick3(left, st[j][0], st[j][1]);
                h[j][1] = P::pick3(st[j][0], st[j][1], right);
            };
            auto step = [&](int s, uint32_t (&cur)[H][CW], uint32_t (&nxt)[H][CW]) {
                uint32_t changed = 0;
                auto fin = [&](int j, int c, uint32_t x) {
                    if constexpr (CLAMP) x = P::clamp(x, m[j][c]);
                    changed |= (x ^ cur[j][c]) & cmask[j][c];
                    nxt[j][c] = x;
                };
#pragma unroll
                for (int c = 0; c < CW; ++c) {
#pragma unroll
                    for (int j = 1; j < H - 1; ++j) fin(j, c, P::pick3(h[j - 1][c], h[j][c], h[j + 1][c]));
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int c = 0; c < CW; ++c) {
                    const uint32_t up0 = __builtin_amdgcn_alignbit(h[H - 1][c], above[c], 16);
                    const uint32_t dnl = __builtin_amdgcn_alignbit(below[c], h[0][c], 16);
                    if constexpr (H == 1) {
                        fin(0, c, P::pick3(up0, h[0][c], dnl));
                    } else {
                        fin(0, c, P::pick3(up0, h[0][c], h[1][c]));
                        fin(H - 1, c, P::pick3(h[H - 2][c], h[H - 1][c], dnl));
                    }
                }
                if (__builtin_amdgcn_ballot_w64(changed != 0)) step_bits |= 1u << s;
                if (s + 1 < busy) {
                    row_pass_of(nxt, 0);
                    if constexpr (H > 1) row_pass_of(nxt, H - 1);
                    publish((s + 1) & 1);
#pragma unroll
                    for (int j = 1; j < H - 1; ++j) row_pass_of(nxt, j);
                }
            };
            int s = 0;
            for (; s + 1 < busy; s += 2) {
                step(s, v, v2);
                step(s + 1, v2, v);
            }
            if (s < busy) {
                step(s, v, v2);
#pragma unroll
                for (int j = 0; j < H; ++j)
#pragma unroll
                    for (int c = 0; c < CW; ++c) v[j][c] = v2[j][c];
            }
        }
    };
    if (wave_has_core)
        run_steps(std::true_type{});
    else
        run_steps(std::false_type{});
    for (int s = busy; s < k; ++s) __syncthreads();

    if constexpr (STAGED) {
        // ---- store the core ----
        // Staged through LDS as well: every lane puts its pixel pairs back into
        // its rows of the staging buffer, then the workgroup writes the core row
        // by row in the widest chunks (16, 8, 4, 2 or 1 bytes) that the core's
        // row starts, its width and the pitch allow, instead of one two-byte
        // store per lane and row.
        {
            uint8_t *sv = stage;
    #pragma unroll
            for (int r = 0; r < RPW; ++r) {
                const int j = r < H ? r : r - H;
                const int sh = r < H ? 0 : 16;
                const uint32_t c0 = (v[j][0] >> sh) & 0xFFu, c1 = (v[j][1] >> sh) & 0xFFu;
                *reinterpret_cast<uint16_t *>(sv + (w * RPW + r) * RX + lane * 2) = (uint16_t)(c0 | (c1 << 8));
            }
            __syncthreads();
            // the core inside the image, in region coordinates
            const int cx0 = halo, cx1 = min(halo + a.core_x, a.width - rx0);
            const int cy0 = halo, cy1 = min(halo + a.core_y, a.height - ry0);
            if (cx1 > cx0 && cy1 > cy0) {
                const int len = cx1 - cx0;
                uint8_t *row0 = dst + (int64_t)(ry0 + cy0) * a.pitch + rx0 + cx0;
                const uintptr_t al = (uintptr_t)row0 | (uintptr_t)a.pitch | (uintptr_t)len | (uintptr_t)cx0;
                // agent-scope stores go out as at most 8-byte atomics
                int G = AGENT_STORES ? 8 : 16;
                while (al & (uintptr_t)(G - 1)) G >>= 1;
                G = __builtin_amdgcn_readfirstlane(G);
                const int per_row = len / G;
                const int n = (cy1 - cy0) * per_row;
                for (int i = threadIdx.x; i < n; i += 64 * NW) {
                    const int r = i / per_row, c = i - r * per_row;
                    const uint8_t *sp = sv + (cy0 + r) * RX + cx0 + c * G;
                    uint8_t *dp = row0 + (int64_t)r * a.pitch + c * G;
                    if constexpr (AGENT_STORES) {
                        // coherent at agent scope on their own, so the release that
                        // publishes the tile finds (almost) nothing to write back
                        if (G == 8)
                            __hip_atomic_store(reinterpret_cast<uint64_t *>(dp), *reinterpret_cast<const uint64_t *>(sp),
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        else if (G == 4)
                            __hip_atomic_store(reinterpret_cast<uint32_t *>(dp), *reinterpret_cast<const uint32_t *>(sp),
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        else if (G == 2)
                            __hip_atomic_store(reinterpret_cast<uint16_t *>(dp), *reinterpret_cast<const uint16_t *>(sp),
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        else
                            __hip_atomic_store(dp, *sp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    } else {
                        if (G == 16)
                            *reinterpret_cast<uint4 *>(dp) = *reinterpret_cast<const uint4 *>(sp);
                        else if (G == 8)
                            *reinterpret_cast<uint2 *>(dp) = *reinterpret_cast<const uint2 *>(sp);
                        else if (G == 4)
                            *reinterpret_cast<uint32_t *>(dp) = *reinterpret_cast<const uint32_t *>(sp);
                        else if (G == 2)
                            *reinterpret_cast<uint16_t *>(dp) = *reinterpret_cast<const uint16_t *>(sp);
                        else
                            *dp = *sp;
                    }
                }
            }
        }
    } else {
        // ---- store the core ----
    #pragma unroll
        for (int r = 0; r < RPW; ++r) {
            const int ry = w * RPW + r;
            const int y = ry0 + ry;
            const bool yok = ry >= halo && ry < halo + a.core_y && y < a.height;
            if (!yok) continue;
            const int j = r < H ? r : r - H;
            const int sh = r < H ? 0 : 16;
            const uint32_t c0 = (v[j][0] >> sh) & 0xFFu, c1 = (v[j][1] >> sh) & 0xFFu;
            const int cx = lane * 2;
            const int x = rx0 + cx;
            uint8_t *p = dst + (int64_t)y * a.pitch + x;
            const bool in0 = cx >= halo && cx < halo + a.core_x && x < a.width;
            const bool in1 = cx + 1 >= halo && cx + 1 < halo + a.core_x && x + 1 < a.width;
            if constexpr (AGENT_STORES) {
                // coherent at agent scope on their own, so the release that
                // publishes the tile finds (almost) nothing to write back
                if (in0 && in1 && (fast || pair_aligned(p))) {
                    __hip_atomic_store(reinterpret_cast<uint16_t *>(p), (uint16_t)(c0 | (c1 << 8)), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                } else {
                    if (in0) __hip_atomic_store(p, (uint8_t)c0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (in1) __hip_atomic_store(p + 1, (uint8_t)c1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            } else if (in0 && in1 && (fast || pair_aligned(p))) {
                *reinterpret_cast<uint16_t *>(p) = (uint16_t)(c0 | (c1 << 8));
            } else {
                if (in0) *p = (uint8_t)c0;
                if (in1) p[1] = (uint8_t)c1;
            }
        }
    }
    return step_bits;
}

template <int G> constexpr int lanes_per_group() { return 64 / G; }

// LDS bytes of the region staging buffer: state and mask of the packed u8
// body when it stages its loads and stores (STAGED); a token size otherwise.
template <typename T, int CW, int RPW, int NW, int G, bool STAGED>
constexpr int stage_bytes() {
    return (STAGED && std::is_same<T, uint8_t>::value && G == 1 && CW == 2 && RPW % 2 == 0)
               ? 2 * (64 * CW) * (NW * RPW)
               : 16;
}

// Plain chains skip the border fence for regions entirely inside the image.
// AGENT_STORES: the core is written with agent-scope stores (packed and
// generic bodies; the persistent kernel, which publishes tiles to other
// workgroups).
template <typename T, int OP, int MODE, bool DETECT, int CW, int RPW, int NW, int G = 1, bool AGENT_STORES = false,
          bool STAGED = false>
__device__ __forceinline__ uint32_t chain_block_dispatch(
    const BlockArgs &a, int rx0, int ry0, typename RegOf<T>::type (*xch)[NW][2 * G][lanes_per_group<G>() * CW],
    uint8_t *stage) {
    constexpr int RX = lanes_per_group<G>() * CW;
    constexpr int RY = NW * RPW * G;
    static_assert(MODE != MODE_MIXED || G == 1, "mixed chains run on one lane group per wave");
    if constexpr (G == 2) {
        if constexpr (MODE == MODE_PLAIN) {
            const bool inside = rx0 >= 0 && ry0 >= 0 && rx0 + RX <= a.width && ry0 + RY <= a.height;
            if (inside) return chain_block_body_g2<T, OP, MODE, false, DETECT, CW, RPW, NW>(a, rx0, ry0, xch);
            return chain_block_body_g2<T, OP, MODE, true, DETECT, CW, RPW, NW>(a, rx0, ry0, xch);
        } else {
            return chain_block_body_g2<T, OP, MODE, true, DETECT, CW, RPW, NW>(a, rx0, ry0, xch);
        }
    } else if constexpr (std::is_same<T, uint8_t>::value && CW == 2 && RPW % 2 == 0) {
        // u8: two rows per register, packed half-precision extrema on encoded pixels
        if constexpr (MODE == MODE_PLAIN || MODE == MODE_MIXED) {
            const bool inside = rx0 >= 0 && ry0 >= 0 && rx0 + RX <= a.width && ry0 + RY <= a.height;
            if (inside) return chain_block_body_pk<OP, MODE, false, DETECT, RPW, NW, AGENT_STORES, STAGED>(a, rx0, ry0, xch, stage);
            return chain_block_body_pk<OP, MODE, true, DETECT, RPW, NW, AGENT_STORES, STAGED>(a, rx0, ry0, xch, stage);
        } else {
            return chain_block_body_pk<OP, MODE, true, DETECT, RPW, NW, AGENT_STORES, STAGED>(a, rx0, ry0, xch, stage);
        }
    } else if constexpr (MODE == MODE_PLAIN || MODE == MODE_MIXED) {
        const bool inside = rx0 >= 0 && ry0 >= 0 && rx0 + RX <= a.width && ry0 + RY <= a.height;
        if (inside) return chain_block_body<T, OP, MODE, false, DETECT, CW, RPW, NW, AGENT_STORES>(a, rx0, ry0, xch);
        return chain_block_body<T, OP, MODE, true, DETECT, CW, RPW, NW, AGENT_STORES>(a, rx0, ry0, xch);
    } else {
        return chain_block_body<T, OP, MODE, true, DETECT, CW, RPW, NW, AGENT_STORES>(a, rx0, ry0, xch);
    }
}

// Tile of a workgroup.  Workgroups are dealt round-robin to the 8 XCDs
// (workgroup b runs on XCD b mod 8), each with its own L2.  XCD x gets the
// band of n/8 consecutive tiles [x n/8, (x+1) n/8): whole tile rows when the
// rows divide evenly, so a tile's left, right and (within the band) upper
// and lower neighbours, whose regions overlap its own, load through the
// same L2.  Measured at 1024^2 u8: 1880 Gpx-steps/s against 1780 in raster
// order, 1800 for 4 x 2 blocks of the tile grid and 1800 for every eighth
// tile row per XCD.  Raster order when n is not a multiple of 8.
__device__ __forceinline__ int xcd_tile(unsigned b, unsigned n) {
    if ((n & 7u) != 0) return (int)b;
    return (int)(b & 7u) * (int)(n >> 3) + (int)(b >> 3);
}

// Change bits of a workgroup go out as one device-scope atomic: the waves
// that hold any first OR them into a word in LDS (set to zero before the
// body's first barrier).  One atomic per wave put up to eight times as
// many atomics on the single change word, where they serialise.
__device__ __forceinline__ void publish_change_bits(uint32_t &wg_bits, uint32_t bits, uint32_t *word) {
    if (bits != 0 && (threadIdx.x & 63) == 0) atomicOr(&wg_bits, bits);
    __syncthreads();
    if (threadIdx.x == 0 && wg_bits != 0) atomicOr(word, wg_bits);
}

template <typename T, int OP, int MODE, bool DETECT, int CW, int RPW, int NW, int G = 1>
__global__ __launch_bounds__(64 * NW) void chain_block_kernel(BlockArgs a) {
    if (DETECT && a.prev_word != nullptr) {
        // The image stopped changing in an earlier launch: nothing to do.
        if (*a.prev_word != a.prev_full) return;
    }
    __shared__ uint32_t wg_bits;
    if (DETECT && threadIdx.x == 0) wg_bits = 0;
    int tile = a.tile0 + xcd_tile(blockIdx.x, gridDim.x);
    BlockArgs b = a;
    if (a.tiles_per_image > 0) {
        // a batch: tiles of image i follow those of image i - 1
        const int img = tile / a.tiles_per_image;
        tile -= img * a.tiles_per_image;
        const int64_t off = (int64_t)img * a.image_stride;
        b.src = static_cast<const T *>(a.src) + off;
        b.mask = a.mask ? static_cast<const T *>(a.mask) + off : nullptr;
        b.dst = static_cast<T *>(a.dst) + off;
    }
    const int tx = tile % a.tiles_x;
    const int ty = tile / a.tiles_x;
    const int rx0 = tx * a.core_x - a.halo;
    const int ry0 = ty * a.core_y - a.halo;
    using R = typename RegOf<T>::type;
    __shared__ __attribute__((aligned(16))) R xch[2][NW][2 * G][lanes_per_group<G>() * CW];
    __shared__ __attribute__((aligned(16))) uint8_t stage[stage_bytes<T, CW, RPW, NW, G, true>()];
    const uint32_t bits =
        chain_block_dispatch<T, OP, MODE, DETECT, CW, RPW, NW, G, false, true>(b, rx0, ry0, xch, stage);
    if constexpr (DETECT) publish_change_bits(wg_bits, bits, a.change_word);
}

}  // namespace geochain
