// operators.hpp -- pixelwise and reduction kernels of the reconstruction-based
// operators of Section 2 (Eq. 6-12).  Each operator is one reconstruction
// (the chain kernels) framed by at most three passes over the image:
//
//   H-maxima, Eq. 6      marker f - h                       (PX_SUB_SCALAR)
//   dome, Eq. 7          f - HMAX_h(f)                      (PX_SUB_IMAGE)
//   hole filling, Eq. 8-9    marker: f on the border B, max f inside
//                                  (extremum_kernel, then PX_BORDER)
//   border objects, Eq. 10-11  marker: f on B, min f inside; then f - rec
//   granulometry, Eq. 17       sum of an opened image (sum_kernel)
//
// Arithmetic is done in the image's dtype: uint8 differences saturate at 0,
// float differences are one IEEE subtraction.  The border B is the first and
// last row and column.
//
// These passes are bound by HBM bandwidth: each reads one or two images and
// writes one, with 16-byte vector accesses when every row start is 16-byte
// aligned, else one element per lane.  The extremum is reduced to one value
// per workgroup (at most PARTIALS_MAX of them); every workgroup of the
// border-marker pass re-reduces those few values itself, so no float atomics
// and no third launch are needed, and the result is independent of the
// reduction order (min/max are exact).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "chain_block.hpp"

namespace geochain {

enum : int { PX_SUB_SCALAR = 0, PX_SUB_IMAGE = 1, PX_BORDER = 2 };

constexpr int PX_THREADS = 256;
constexpr int PARTIALS_MAX = 1024;

template <typename T> struct PixelArgs {
    const T *a;          // f
    const T *b;          // second operand of PX_SUB_IMAGE
    T *out;              // result image (PX_*) or PARTIALS_MAX partials (extremum)
    const T *partials;   // PX_BORDER: per-workgroup extrema of f
    int32_t n_partials;
    T h;                 // PX_SUB_SCALAR
    int32_t width, height;
    int64_t pitch;           // elements
    int64_t chunks_per_row;  // ceil(width / V)
    int64_t n_chunks;        // height * chunks_per_row
};

template <typename T> __device__ __forceinline__ T sub_in_dtype(T a, T b) { return a - b; }
template <> __device__ __forceinline__ uint8_t sub_in_dtype<uint8_t>(uint8_t a, uint8_t b) {
    return a > b ? (uint8_t)(a - b) : (uint8_t)0;
}

// better(OP): max for OP_DILATE, min for OP_ERODE.
template <int OP, typename T> __device__ __forceinline__ T px_better(T a, T b) {
    if constexpr (OP == OP_DILATE) return a > b ? a : b;
    else return a < b ? a : b;
}

template <int OP, typename T> __device__ __forceinline__ T px_identity() {
    using R = typename RegOf<T>::type;
    return (T)Bounds<R, OP>::bottom();
}

// Extremum over the whole workgroup; every thread gets the result.
template <int OP, typename T> __device__ __forceinline__ T block_extremum(T v) {
    __shared__ T red[PX_THREADS];
    red[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int s = PX_THREADS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = px_better<OP>(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    const T r = red[0];
    __syncthreads();
    return r;
}

template <typename T, int VEC> union Chunk {
    uint4 v;
    T e[VEC];
};

// Visits every pixel chunk (V consecutive pixels of one row) of the image.
// fn(x0, y, off, nvalid) handles one chunk; VEC chunks are whole and
// 16-byte aligned when nvalid == V.
template <bool VEC, typename T, typename Fn>
__device__ __forceinline__ void for_chunks(const PixelArgs<T> &p, Fn fn) {
    constexpr int V = VEC ? 16 / (int)sizeof(T) : 1;
    const int64_t stride = (int64_t)gridDim.x * PX_THREADS;
    for (int64_t c = (int64_t)blockIdx.x * PX_THREADS + threadIdx.x; c < p.n_chunks; c += stride) {
        const int64_t y = c / p.chunks_per_row;
        const int64_t x0 = (c - y * p.chunks_per_row) * V;
        const int64_t left = p.width - x0;
        fn(x0, y, y * p.pitch + x0, left < V ? (int)left : V);
    }
}

// Per-workgroup extremum of f -> p.out[blockIdx.x].
template <typename T, int OP, bool VEC>
__global__ __launch_bounds__(PX_THREADS) void extremum_kernel(PixelArgs<T> p) {
    constexpr int V = VEC ? 16 / (int)sizeof(T) : 1;
    T acc = px_identity<OP, T>();
    for_chunks<VEC>(p, [&](int64_t, int64_t, int64_t off, int nvalid) {
        if (VEC && nvalid == V) {
            Chunk<T, V> c;
            c.v = *reinterpret_cast<const uint4 *>(p.a + off);
#pragma unroll
            for (int j = 0; j < V; ++j) acc = px_better<OP>(acc, c.e[j]);
        } else {
            for (int j = 0; j < nvalid; ++j) acc = px_better<OP>(acc, p.a[off + j]);
        }
    });
    acc = block_extremum<OP>(acc);
    if (threadIdx.x == 0) p.out[blockIdx.x] = acc;
}

template <typename T, int KIND, int OP>
__device__ __forceinline__ T pixel_value(const PixelArgs<T> &p, T a, T b, T ext, int64_t x, int64_t y) {
    if constexpr (KIND == PX_SUB_SCALAR) return sub_in_dtype(a, p.h);
    else if constexpr (KIND == PX_SUB_IMAGE) return sub_in_dtype(a, b);
    else {
        const bool border = x == 0 || y == 0 || x == p.width - 1 || y == p.height - 1;
        return border ? a : ext;
    }
}

// out = pixelwise function of f (and b): the marker images and the final
// differences of the operators.  out may equal a or b (each pixel is read
// before it is written, by the same lane).
template <typename T, int KIND, int OP, bool VEC>
__global__ __launch_bounds__(PX_THREADS) void pixel_kernel(PixelArgs<T> p) {
    constexpr int V = VEC ? 16 / (int)sizeof(T) : 1;
    T ext = px_identity<OP, T>();
    if constexpr (KIND == PX_BORDER) {
        T acc = px_identity<OP, T>();
        for (int i = threadIdx.x; i < p.n_partials; i += PX_THREADS) acc = px_better<OP>(acc, p.partials[i]);
        ext = block_extremum<OP>(acc);
    }
    for_chunks<VEC>(p, [&](int64_t x0, int64_t y, int64_t off, int nvalid) {
        if (VEC && nvalid == V) {
            Chunk<T, V> ca, cb, co;
            ca.v = *reinterpret_cast<const uint4 *>(p.a + off);
            if constexpr (KIND == PX_SUB_IMAGE) cb.v = *reinterpret_cast<const uint4 *>(p.b + off);
#pragma unroll
            for (int j = 0; j < V; ++j)
                co.e[j] = pixel_value<T, KIND, OP>(p, ca.e[j], KIND == PX_SUB_IMAGE ? cb.e[j] : T(0), ext,
                                                   x0 + j, y);
            *reinterpret_cast<uint4 *>(p.out + off) = co.v;
        } else {
            for (int j = 0; j < nvalid; ++j) {
                const T b = KIND == PX_SUB_IMAGE ? p.b[off + j] : T(0);
                p.out[off + j] = pixel_value<T, KIND, OP>(p, p.a[off + j], b, ext, x0 + j, y);
            }
        }
    });
}

// ---------------------------------------------------------------------------
// Sum of an image (granulometric function, Eq. 17) in float64, in a fixed
// order: each thread adds its chunks in turn, each workgroup reduces by a
// fixed tree into one partial, and sum_partials_kernel adds those
// partials in a fixed tree as well (the partials of several images at once,
// one workgroup each), so repeated calls give identical bits.
// Integer-valued images sum exactly (below 2^53).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double block_sum(double v) {
    __shared__ double red[PX_THREADS];
    red[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int s = PX_THREADS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

template <typename T, bool VEC>
__global__ __launch_bounds__(PX_THREADS) void sum_kernel(PixelArgs<T> p, double *partials) {
    constexpr int V = VEC ? 16 / (int)sizeof(T) : 1;
    double acc = 0.0;
    for_chunks<VEC>(p, [&](int64_t, int64_t, int64_t off, int nvalid) {
        if (VEC && nvalid == V) {
            Chunk<T, V> c;
            c.v = *reinterpret_cast<const uint4 *>(p.a + off);
#pragma unroll
            for (int j = 0; j < V; ++j) acc += (double)c.e[j];
        } else {
            for (int j = 0; j < nvalid; ++j) acc += (double)p.a[off + j];
        }
    });
    acc = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = acc;
}

// Workgroup b: out[b] = sum of partials[b * stride .. b * stride + n[b]).
constexpr int SUMS_PER_LAUNCH = 64;
struct PartialCounts {
    int n[SUMS_PER_LAUNCH];
};
__global__ __launch_bounds__(PX_THREADS) void sum_partials_kernel(const double *partials, int64_t stride,
                                                                  PartialCounts counts, double *out) {
    const double *p = partials + blockIdx.x * stride;
    const int n = counts.n[blockIdx.x];
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += PX_THREADS) acc += p[i];
    acc = block_sum(acc);
    if (threadIdx.x == 0) out[blockIdx.x] = acc;
}

// ---------------------------------------------------------------------------
// Value scan: bit 0 of flags[0] is set if some pixel is a NaN, bit 1 if some
// pixel is an infinity.  The tests look at the bit patterns (exponent all
// ones; mantissa nonzero for NaN, zero for an infinity), so they hold
// whatever the compiler assumes about NaNs.  Findings are rare, so a thread
// with one ORs it in directly.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t value_class(float x) {
    const uint32_t a = __builtin_bit_cast(uint32_t, x) & 0x7FFFFFFFu;
    return a > 0x7F800000u ? 1u : (a == 0x7F800000u ? 2u : 0u);
}
__device__ __forceinline__ uint32_t value_class(double x) {
    const uint64_t a = __builtin_bit_cast(uint64_t, x) & 0x7FFFFFFFFFFFFFFFull;
    return a > 0x7FF0000000000000ull ? 1u : (a == 0x7FF0000000000000ull ? 2u : 0u);
}

template <typename T, bool VEC>
__global__ __launch_bounds__(PX_THREADS) void value_scan_kernel(PixelArgs<T> p, uint32_t *flags) {
    constexpr int V = VEC ? 16 / (int)sizeof(T) : 1;
    uint32_t bits = 0;
    for_chunks<VEC>(p, [&](int64_t, int64_t, int64_t off, int nvalid) {
        if (VEC && nvalid == V) {
            Chunk<T, V> c;
            c.v = *reinterpret_cast<const uint4 *>(p.a + off);
#pragma unroll
            for (int j = 0; j < V; ++j) bits |= value_class(c.e[j]);
        } else {
            for (int j = 0; j < nvalid; ++j) bits |= value_class(p.a[off + j]);
        }
    });
    if (bits != 0) atomicOr(flags, bits);
}

}  // namespace geochain
