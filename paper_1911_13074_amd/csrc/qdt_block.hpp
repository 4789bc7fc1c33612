// qdt_block.hpp -- temporal-blocked kernels of the quasi-distance transform
// (Section 2, Eq. 13-15; Algorithm 6).
//
// Phase QDT_ERODE runs the chain of plain 3x3 erosions eps_j = eps_1(eps_{j-1})
// and, for every pixel, keeps the largest residual eps_{j-1} - eps_j seen so
// far (r, in the image dtype) and the first erosion index j that reached it
// (d, int32): a later erosion replaces them only with a strictly larger
// residual.  This is the bookkeeping of Algorithm 6; the conditional update
// becomes a compare and two selects per pixel and step, in registers.
//
// Phase QDT_ETA applies eta(g) = min(g, eps_1(g) + 1) to the int32 distance
// image (Eq. 14: where g exceeds its window minimum by more than 1 it drops
// to that minimum + 1, else it stays; the window contains g itself, so this
// is exactly the min).
//
// Both phases reuse the register layout of chain_block.hpp (u8 erosions its
// packed two-rows-per-register form, qdt_erode_body_pk): a workgroup of
// NW waves holds a region of (64 CW) x (NW RPW) pixels in registers, runs k
// steps on chip and writes the k-pixel-inset core.  The row pass takes its
// neighbour columns from adjacent lanes by DPP; the edge rows of each wave go
// through LDS, one barrier per step.  Pixels outside the image are fenced to
// the neutral value every step (the clipped window of Section 2).  Each step
// ORs "some core pixel changed" into a per-launch word, and a launch whose
// predecessor saw a step without change exits at once (both chains stop at
// their first step that changes nothing: after it every residual is 0 and
// eta has reached its limit).
//
// The residual and distance images are read and written only at core pixels,
// in place: cores of different workgroups are disjoint and the halo never
// needs them.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "chain_block.hpp"

namespace geochain {

enum : int { QDT_ERODE = 0, QDT_ETA = 1 };

// Register type and the value outside the image (never wins a minimum).
template <typename T> struct QdtReg;
template <> struct QdtReg<uint8_t> {
    using type = uint32_t;
    static __device__ __forceinline__ uint32_t neutral() { return 255u; }
};
template <> struct QdtReg<float> {
    using type = float;
    static __device__ __forceinline__ float neutral() { return __builtin_inff(); }
};
template <> struct QdtReg<double> {
    using type = double;
    static __device__ __forceinline__ double neutral() { return __builtin_inf(); }
};
// eta state: non-negative int32 distances handled as unsigned.
template <> struct QdtReg<uint32_t> {
    using type = uint32_t;
    static __device__ __forceinline__ uint32_t neutral() { return 0xFFFFFFFFu; }
};

__device__ __forceinline__ uint32_t qdt_to_reg(uint8_t v) { return v; }
__device__ __forceinline__ uint32_t qdt_to_reg(uint32_t v) { return v; }
__device__ __forceinline__ float qdt_to_reg(float v) { return v; }
__device__ __forceinline__ double qdt_to_reg(double v) { return v; }
__device__ __forceinline__ void qdt_from_reg(uint8_t *p, uint32_t v) { *p = (uint8_t)v; }
__device__ __forceinline__ void qdt_from_reg(uint32_t *p, uint32_t v) { *p = v; }
__device__ __forceinline__ void qdt_from_reg(float *p, float v) { *p = v; }
__device__ __forceinline__ void qdt_from_reg(double *p, double v) { *p = v; }

__device__ __forceinline__ uint32_t qdt_min(uint32_t a, uint32_t b) { return a < b ? a : b; }
__device__ __forceinline__ float qdt_min(float a, float b) { return __builtin_fminf(a, b); }
__device__ __forceinline__ double qdt_min(double a, double b) { return __builtin_fmin(a, b); }

struct QdtArgs {
    BlockArgs b;       // state in (src) / out (dst), shape, k, halo, core, change words
    void *res;         // QDT_ERODE: residual image r (image dtype), core pixels in place
    int32_t *dist;     // QDT_ERODE: distance image d, core pixels in place
    int32_t step0;     // QDT_ERODE: erosions applied before this launch (0: r, d start at 0)
};

// T: image dtype for QDT_ERODE, uint32_t (the distances) for QDT_ETA.
template <typename T, int PHASE, bool FENCE, int CW, int RPW, int NW>
__device__ __forceinline__ uint32_t qdt_block_body(const QdtArgs &qa, int rx0, int ry0,
                                                   typename QdtReg<T>::type (*xch)[NW][2][64 * CW]) {
    using R = typename QdtReg<T>::type;
    const BlockArgs &a = qa.b;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const T *src = static_cast<const T *>(a.src);
    T *dst = static_cast<T *>(a.dst);
    const int k = a.k;
    const int halo = a.halo;
    constexpr bool TRACK = PHASE == QDT_ERODE;

    // Columns of this lane inside the image / inside the core; rows are
    // uniform per wave and tested per row.
    bool col_img[CW];
    bool col_core[CW];
    uint64_t col_core_mask[CW];
#pragma unroll
    for (int c = 0; c < CW; ++c) {
        const int cx = lane * CW + c;
        const int x = rx0 + cx;
        col_img[c] = (unsigned)x < (unsigned)a.width;
        col_core[c] = cx >= halo && cx < halo + a.core_x && x < a.width;
        col_core_mask[c] = __builtin_amdgcn_ballot_w64(col_core[c]);
    }
    auto row_img = [&](int r) { return (unsigned)(ry0 + w * RPW + r) < (unsigned)a.height; };
    auto row_core = [&](int r) {
        const int ry = w * RPW + r;
        return ry >= halo && ry < halo + a.core_y && ry0 + ry < a.height;
    };

    // ---- load the region's state; r and d at core pixels ----
    R v[RPW][CW];
    R rr[TRACK ? RPW : 1][TRACK ? CW : 1];
    int32_t dd[TRACK ? RPW : 1][TRACK ? CW : 1];
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
        const int y = ry0 + w * RPW + r;
        const bool yin = row_img(r);
        const bool ycore = row_core(r);
#pragma unroll
        for (int c = 0; c < CW; ++c) {
            const int x = rx0 + lane * CW + c;
            const int64_t off = (int64_t)y * a.pitch + x;
            v[r][c] = (yin && col_img[c]) ? qdt_to_reg(src[off]) : QdtReg<T>::neutral();
            if constexpr (TRACK) {
                const bool load = ycore && col_core[c] && qa.step0 > 0;
                rr[r][c] = load ? qdt_to_reg(static_cast<const T *>(qa.res)[off]) : R(0);
                dd[r][c] = load ? qa.dist[off] : 0;
            }
        }
    }

    // Rows still needed after step s lie within k-1-s of the core (plus one
    // for the row pass); a wave past that band only takes the barriers.
    const int busy_a = w * RPW + RPW - (halo - k);
    const int busy_b = halo + a.core_y + k - w * RPW;
    const int busy = __builtin_amdgcn_readfirstlane(max(0, min(k, min(busy_a, busy_b))));
    const bool wave_has_core = w * RPW + RPW > halo && w * RPW < halo + a.core_y;
    uint32_t step_bits = 0;

    auto run_steps = [&](auto core_tag) {
        constexpr bool CORE = decltype(core_tag)::value;
        for (int s = 0; s < busy; ++s) {
            // ---- row pass ----
            R h[RPW][CW];
#pragma unroll
            for (int r = 0; r < RPW; ++r) {
                const R left = lane_shift<DPP_WAVE_SHR1>(v[r][CW - 1]);
                const R right = lane_shift<DPP_WAVE_SHL1>(v[r][0]);
                if constexpr (CW == 1) {
                    h[r][0] = qdt_min(qdt_min(left, v[r][0]), right);
                } else {
                    const R t = qdt_min(v[r][0], v[r][1]);
                    h[r][0] = qdt_min(t, left);
                    h[r][1] = qdt_min(t, right);
                }
            }
            // ---- edge rows through LDS ----
            const int par = s & 1;
#pragma unroll
            for (int c = 0; c < CW; ++c) {
                xch[par][w][0][lane * CW + c] = h[0][c];
                xch[par][w][1][lane * CW + c] = h[RPW - 1][c];
            }
            __syncthreads();
            const int wa = w > 0 ? w - 1 : NW - 1;
            const int wb = w < NW - 1 ? w + 1 : 0;
            R above[CW], below[CW];
#pragma unroll
            for (int c = 0; c < CW; ++c) {
                above[c] = xch[par][wa][1][lane * CW + c];
                below[c] = xch[par][wb][0][lane * CW + c];
            }
            // ---- column pass, phase update ----
            const int32_t j = qa.step0 + s + 1;
            uint64_t changed = 0;
#pragma unroll
            for (int r = 0; r < RPW; ++r) {
                const bool yin = !FENCE || row_img(r);
                const uint64_t row_mask = CORE && row_core(r) ? ~0ull : 0ull;
#pragma unroll
                for (int c = 0; c < CW; ++c) {
                    const R up = r == 0 ? above[c] : h[r - 1][c];
                    const R dn = r == RPW - 1 ? below[c] : h[r + 1][c];
                    R nv = qdt_min(qdt_min(up, h[r][c]), dn);
                    if constexpr (PHASE == QDT_ETA) nv = qdt_min(v[r][c], nv + 1u);
                    if constexpr (FENCE) nv = (yin && col_img[c]) ? nv : QdtReg<T>::neutral();
                    if constexpr (CORE) {
                        if constexpr (TRACK) {
                            const R res = v[r][c] - nv;   // >= 0: the window holds the pixel
                            const bool upd = res > rr[r][c];
                            rr[r][c] = upd ? res : rr[r][c];
                            dd[r][c] = upd ? j : dd[r][c];
                        }
                        changed |= __builtin_amdgcn_ballot_w64(nv != v[r][c]) & col_core_mask[c] & row_mask;
                    }
                    v[r][c] = nv;
                }
            }
            if constexpr (CORE) {
                if (changed) step_bits |= 1u << s;
            }
        }
    };
    if (wave_has_core)
        run_steps(std::true_type{});
    else
        run_steps(std::false_type{});
    for (int s = busy; s < k; ++s) __syncthreads();

    // ---- store the core: state, and r, d ----
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
        if (!row_core(r)) continue;
        const int y = ry0 + w * RPW + r;
#pragma unroll
        for (int c = 0; c < CW; ++c) {
            if (!col_core[c]) continue;
            const int64_t off = (int64_t)y * a.pitch + rx0 + lane * CW + c;
            qdt_from_reg(dst + off, v[r][c]);
            if constexpr (TRACK) {
                qdt_from_reg(static_cast<T *>(qa.res) + off, rr[r][c]);
                qa.dist[off] = dd[r][c];
            }
        }
    }
    return step_bits;
}

// ---------------------------------------------------------------------------
// u8 erosion phase with two rows per register (the packed layout of
// chain_block_body_pk: register j holds rows j and j + RPW/2, each pixel p
// encoded as the binary16 number 1024 + p).  The residual of a step is the
// packed 16-bit difference of the encodings, p_before - p_after (the window
// holds the pixel, so it is >= 0).  Within a launch, the largest residual
// and the first step reaching it are tracked together as the running
// maximum of the 16-bit key residual * 256 + (255 - s): a larger residual
// wins, and among equal residuals the earlier step.  At the end of the
// launch each core pixel merges that maximum into the stored r and d with
// the same strict rule (a launch's best replaces them only if larger), which
// gives what the step-by-step update gives.  A step changed the core iff
// some core residual is nonzero.
// ---------------------------------------------------------------------------
template <bool FENCE, int RPW, int NW>
__device__ __forceinline__ uint32_t qdt_erode_body_pk(const QdtArgs &qa, int rx0, int ry0,
                                                      uint32_t (*xch)[NW][2][128]) {
    static_assert(RPW % 2 == 0, "two rows per register");
    constexpr int H = RPW / 2;
    constexpr int CW = 2;
    using P = PackedPick<OP_ERODE>;
    typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
    const BlockArgs &a = qa.b;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint8_t *src = static_cast<const uint8_t *>(a.src);
    uint8_t *dst = static_cast<uint8_t *>(a.dst);
    const int k = a.k;
    const int halo = a.halo;
    constexpr uint32_t NEUTRAL = 255u;  // never wins a minimum

    uint32_t v[H][CW];
    uint32_t m[FENCE ? H : 1][CW];   // 0 inside the image, 255 outside: max(x, m) fences the border
    const bool fast = !FENCE && (a.pitch & 1) == 0 && pair_aligned(src);
    if (fast) {
        const int64_t base = (int64_t)(ry0 + w * RPW) * a.pitch + rx0 + lane * 2;
#pragma unroll
        for (int j = 0; j < H; ++j) {
            const uint32_t lo = *reinterpret_cast<const uint16_t *>(src + base + j * a.pitch);
            const uint32_t hi = *reinterpret_cast<const uint16_t *>(src + base + (j + H) * a.pitch);
            v[j][0] = pack_rows(lo & 0xFFu, hi & 0xFFu);
            v[j][1] = pack_rows(lo >> 8, hi >> 8);
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
                    vv[half] = in ? (uint32_t)src[(int64_t)y * a.pitch + x] : NEUTRAL;
                    mm[half] = in ? 0u : NEUTRAL;
                }
                v[j][c] = pack_rows(vv[0], vv[1]);
                if constexpr (FENCE) m[j][c] = pack_rows(mm[0], mm[1]);
            }
        }
    }

    // 16-bit core masks per register half and column (loop invariant)
    uint32_t cmask[H][CW];
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
    uint32_t key[H][CW];
#pragma unroll
    for (int j = 0; j < H; ++j)
#pragma unroll
        for (int c = 0; c < CW; ++c) key[j][c] = 0;

    const int busy_a = w * RPW + RPW - (halo - k);
    const int busy_b = halo + a.core_y + k - w * RPW;
    const int busy = __builtin_amdgcn_readfirstlane(max(0, min(k, min(busy_a, busy_b))));
    const bool wave_has_core = w * RPW + RPW > halo && w * RPW < halo + a.core_y;
    uint32_t step_bits = 0;

    auto run_steps = [&](auto core_tag) {
        constexpr bool CORE = decltype(core_tag)::value;
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
        uint32_t any = 0;
        auto finish = [&](int j, int c, uint32_t x, uint32_t (&nv)[H][CW], int s) {
            if constexpr (FENCE) x = P::clamp(x, m[j][c]);
            if constexpr (CORE) {
                const uint32_t res =
                    __builtin_bit_cast(uint32_t, __builtin_bit_cast(u16x2, v[j][c]) - __builtin_bit_cast(u16x2, x));
                // halves res * 256 + (255 - s): each residual byte moves above
                // the step tag (core residuals are below 256)
                const uint32_t kk = __builtin_amdgcn_perm(res, (uint32_t)(255 - s), 0x06000400u);
                key[j][c] = __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(u16x2, key[j][c]),
                                                                                   __builtin_bit_cast(u16x2, kk)));
                any |= res & cmask[j][c];
            }
            nv[j][c] = x;
        };

#pragma unroll
        for (int j = 0; j < H; ++j) row_pass(j);
        publish(0);
        for (int s = 0; s < busy; ++s) {
            uint32_t nv[H][CW];
            any = 0;
#pragma unroll
            for (int c = 0; c < CW; ++c) {
#pragma unroll
                for (int j = 1; j < H - 1; ++j) finish(j, c, P::pick3(h[j - 1][c], h[j][c], h[j + 1][c]), nv, s);
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int c = 0; c < CW; ++c) {
                const uint32_t up0 = __builtin_amdgcn_alignbit(h[H - 1][c], above[c], 16);
                const uint32_t dnl = __builtin_amdgcn_alignbit(below[c], h[0][c], 16);
                if constexpr (H == 1) {
                    finish(0, c, P::pick3(up0, h[0][c], dnl), nv, s);
                } else {
                    finish(0, c, P::pick3(up0, h[0][c], h[1][c]), nv, s);
                    finish(H - 1, c, P::pick3(h[H - 2][c], h[H - 1][c], dnl), nv, s);
                }
            }
#pragma unroll
            for (int j = 0; j < H; ++j)
#pragma unroll
                for (int c = 0; c < CW; ++c) v[j][c] = nv[j][c];
            if constexpr (CORE) {
                if (__builtin_amdgcn_ballot_w64(any != 0)) step_bits |= 1u << s;
            }
            if (s + 1 < busy) {
                row_pass(0);
                if constexpr (H > 1) row_pass(H - 1);
                publish((s + 1) & 1);
#pragma unroll
                for (int j = 1; j < H - 1; ++j) row_pass(j);
            }
        }
    };
    if (wave_has_core)
        run_steps(std::true_type{});
    else
        run_steps(std::false_type{});
    for (int s = busy; s < k; ++s) __syncthreads();

    // ---- store the core: state; merge the launch's best into r and d ----
    uint8_t *res_img = static_cast<uint8_t *>(qa.res);
#pragma unroll
    for (int r = 0; r < RPW; ++r) {
        const int ry = w * RPW + r;
        const int y = ry0 + ry;
        if (!(ry >= halo && ry < halo + a.core_y && y < a.height)) continue;
        const int j = r < H ? r : r - H;
        const int sh = r < H ? 0 : 16;
#pragma unroll
        for (int c = 0; c < CW; ++c) {
            const int cx = lane * CW + c;
            const int x = rx0 + cx;
            if (!(cx >= halo && cx < halo + a.core_x && x < a.width)) continue;
            const int64_t off = (int64_t)y * a.pitch + x;
            dst[off] = (uint8_t)(v[j][c] >> sh);
            const uint32_t kk = (key[j][c] >> sh) & 0xFFFFu;
            const uint32_t best = kk >> 8;
            const uint32_t prev = qa.step0 > 0 ? (uint32_t)res_img[off] : 0u;
            if (best > prev) {
                res_img[off] = (uint8_t)best;
                qa.dist[off] = qa.step0 + (255 - (int32_t)(kk & 0xFFu)) + 1;
            } else if (qa.step0 == 0) {
                res_img[off] = 0;
                qa.dist[off] = 0;
            }
        }
    }
    return step_bits;
}

template <typename T, int PHASE, int CW, int RPW, int NW>
__global__ __launch_bounds__(64 * NW) void qdt_block_kernel(QdtArgs qa) {
    const BlockArgs &a = qa.b;
    if (a.prev_word != nullptr) {
        // an earlier launch already saw a step without change
        if (*a.prev_word != a.prev_full) return;
    }
    __shared__ uint32_t wg_bits;
    if (threadIdx.x == 0) wg_bits = 0;
    const int tile = a.tile0 + xcd_tile(blockIdx.x, gridDim.x);
    const int rx0 = (tile % a.tiles_x) * a.core_x - a.halo;
    const int ry0 = (tile / a.tiles_x) * a.core_y - a.halo;
    using R = typename QdtReg<T>::type;
    __shared__ __attribute__((aligned(16))) R xch[2][NW][2][64 * CW];
    constexpr int RX = 64 * CW, RY = NW * RPW;
    const bool inside = rx0 >= 0 && ry0 >= 0 && rx0 + RX <= a.width && ry0 + RY <= a.height;
    uint32_t bits;
    if constexpr (std::is_same<T, uint8_t>::value && PHASE == QDT_ERODE && CW == 2 && RPW % 2 == 0) {
        bits = inside ? qdt_erode_body_pk<false, RPW, NW>(qa, rx0, ry0, xch)
                      : qdt_erode_body_pk<true, RPW, NW>(qa, rx0, ry0, xch);
    } else {
        bits = inside ? qdt_block_body<T, PHASE, false, CW, RPW, NW>(qa, rx0, ry0, xch)
                      : qdt_block_body<T, PHASE, true, CW, RPW, NW>(qa, rx0, ry0, xch);
    }
    publish_change_bits(wg_bits, bits, a.change_word);
}

}  // namespace geochain
