/*
 * geochain.h -- C ABI of the MI355X (gfx950) library for long chains of
 * elementary 3x3 geodesic dilations and erosions.
 *
 * Method: Zlaus & Mongus, "Efficient method for parallel computation of
 * geodesic transformation on CPU" (2019).  Definitions used throughout:
 *
 *   image       f : P -> R, P = {0..X-1} x {0..Y-1} (Section 2); stored
 *               row-major, pixel (x, y) at element offset y * pitch + x.
 *   window      the 3x3 square w_1(p), clipped to P (Section 2).
 *   delta_1, eps_1   max / min over the window (Eq. 1-2).
 *   geodesic step    delta_1^m(f) = min(delta_1(f), m),
 *                    eps_1^m(f)   = max(eps_1(f), m)         (Eq. 3).
 *   chain of n       n-fold composition of the step           (Eq. 4).
 *   reconstruction   the limit of the chain as n grows         (Eq. 5),
 *                    reached at the first step that changes no pixel
 *                    (convergence test of Section 3.7, Algorithm 5).
 *
 * Every result is exact: the steps only select existing values, so u8,
 * f32 and f64 results are bit-identical to the definitions.  NaN inputs are
 * outside the definitions and give unspecified (but memory-safe) results;
 * -0.0 and +0.0 compare equal and either may be returned.
 *
 * Conventions for every entry point:
 *   - Image pointers are DEVICE pointers, owned by the caller.  The library
 *     owns only its internal workspaces (cached per device and stream) and
 *     gc_plan objects.
 *   - shape.pitch is in elements and must be >= shape.width; marker, mask
 *     and out share the shape.  width or height 0 is a valid empty image.
 *   - out may equal marker (in place, as the paper's filters run in place,
 *     Section 3.3).  out must not overlap mask (GC_ERR_ALIAS), and a partial
 *     overlap of out with marker is rejected too.
 *   - Work is enqueued on hip_stream (a hipStream_t; NULL = the null
 *     stream) and is asynchronous unless the entry point says otherwise.
 *   - The return value is GC_OK or a negative gc_status.  Arguments are
 *     validated before any HIP call; on error nothing is enqueued.
 *     gc_last_error() gives a detail message for the calling thread.
 *   - Calls that run concurrently on different streams are safe; each
 *     (device, stream) pair has its own workspace.
 */
#ifndef GEOCHAIN_H
#define GEOCHAIN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { GC_U8 = 0, GC_F32 = 1, GC_F64 = 2 } gc_dtype;
typedef enum { GC_DILATE = 0, GC_ERODE = 1 } gc_op;

typedef enum {
    GC_OK = 0,
    GC_ERR_INVALID_ARG = -1,
    GC_ERR_UNSUPPORTED = -2,
    GC_ERR_ALIAS = -3,
    GC_ERR_NO_MEMORY = -4,
    GC_ERR_HIP = -5,
    GC_ERR_NOT_CONVERGED = -6
} gc_status;

typedef struct {
    int64_t width;   /* X, pixels per row            */
    int64_t height;  /* Y, rows                      */
    int64_t pitch;   /* elements between row starts  */
} gc_shape;

/* Library version as major*10000 + minor*100 + patch. */
int gc_version(void);

/* Human-readable name of a gc_status value (static string). */
const char *gc_status_string(int status);

/* Detail message of the last error on the calling thread ("" if none). */
const char *gc_last_error(void);

/* ---------------------------------------------------------------------
 * Geodesic chains (Eq. 3-4).
 *
 * out = (delta_1^mask)^n_steps (marker)   for gc_geodesic_dilate_chain,
 * out = (eps_1^mask)^n_steps (marker)     for gc_geodesic_erode_chain.
 *
 * n_steps >= 0; n_steps = 0 copies marker to out unchanged (no clamp).
 * marker need not lie below (above) the mask: the clamp applies from the
 * first step on.
 * ------------------------------------------------------------------- */
int gc_geodesic_dilate_chain(gc_dtype dtype, const void *marker, const void *mask,
                             void *out, gc_shape shape, int64_t n_steps,
                             void *hip_stream);
int gc_geodesic_erode_chain(gc_dtype dtype, const void *marker, const void *mask,
                            void *out, gc_shape shape, int64_t n_steps,
                            void *hip_stream);

/* ---------------------------------------------------------------------
 * Plain chains (Eq. 1-2 iterated): n_steps 3x3 dilations (erosions),
 * equal to one (2 n_steps + 1)^2 window clipped to the image.
 * in may equal out.
 * ------------------------------------------------------------------- */
int gc_dilate_chain(gc_dtype dtype, const void *in, void *out, gc_shape shape,
                    int64_t n_steps, void *hip_stream);
int gc_erode_chain(gc_dtype dtype, const void *in, void *out, gc_shape shape,
                   int64_t n_steps, void *hip_stream);

/* ---------------------------------------------------------------------
 * Reconstruction (Eq. 5): repeat the geodesic step until one application
 * changes no pixel.
 *
 * max_steps caps the number of applications (< 0: no cap).  On return,
 * *steps_out (host pointer, may be NULL) holds the number of applications
 * that changed at least one pixel, so that out equals the chain of that
 * length.  These calls SYNCHRONISE hip_stream (the number of steps is
 * data-dependent).  GC_ERR_NOT_CONVERGED: the cap was reached while the
 * image still changed; out then holds the chain of length max_steps and
 * *steps_out = max_steps.
 * ------------------------------------------------------------------- */
int gc_reconstruct_by_dilation(gc_dtype dtype, const void *marker, const void *mask,
                               void *out, gc_shape shape, int64_t max_steps,
                               int64_t *steps_out, void *hip_stream);
int gc_reconstruct_by_erosion(gc_dtype dtype, const void *marker, const void *mask,
                              void *out, gc_shape shape, int64_t max_steps,
                              int64_t *steps_out, void *hip_stream);

/* ---------------------------------------------------------------------
 * Tuning hook: override the temporal-block depth (steps fused per launch)
 * and the tile family used by the chain kernels.  block_steps = 0 and
 * tile = -1 restore the built-in choice.  Process-wide; intended for the
 * autotuner and for tests that sweep launch shapes.
 * ------------------------------------------------------------------- */
int gc_set_tuning(int32_t block_steps, int32_t tile);

/* ---------------------------------------------------------------------
 * Measurement hook.  While enabled (on != 0), every kernel launch made by
 * the entry points above is bracketed by two HIP events recorded on the
 * launch stream.  gc_profile_read waits for the last event, returns the sum
 * of the bracketed times in milliseconds (*kernel_ms), the number of
 * bracketed launches (*launches) and the steps those launches advanced
 * (*steps), then clears the record.  Disabling also clears it.  Intended
 * for benchmarks: recording events between launches costs a little time.
 * ------------------------------------------------------------------- */
int gc_profile_enable(int on);
int gc_profile_read(double *kernel_ms, int64_t *launches, int64_t *steps);

#ifdef __cplusplus
}
#endif

#endif /* GEOCHAIN_H */
