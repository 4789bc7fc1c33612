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
 * On these the library builds the operators of Section 2: H-maxima, dome
 * extraction, hole filling, removal of border objects and opening by
 * reconstruction (Eq. 6-12), the quasi-distance transform (Eq. 13-15,
 * Algorithm 6), granulometry, pattern spectrum and alternating sequential
 * filters (Eq. 16-20); plus, beyond the paper, batches of chains in one
 * persistent launch and the gradient of a chain.
 *
 * Chains, reconstructions and plain windows are exact: the steps only
 * select existing values, so u8, f32 and f64 results are bit-identical to
 * the definitions.  Where an operator subtracts, it does so once in the
 * image's dtype, as stated at its declaration.  NaN inputs are
 * outside the definitions and give unspecified (but memory-safe) results;
 * -0.0 and +0.0 compare equal and either may be returned.
 *
 * Conventions for every entry point:
 *   - Image pointers are DEVICE pointers, owned by the caller.  The library
 *     owns only its internal workspaces (cached per device and stream) and
 *     gc_plan objects.
 *   - shape.pitch is in elements and must be >= shape.width; marker, mask
 *     and out share the shape.  width or height 0 is a valid empty image.
 *     Sides above 2^25 or more than 2^36 pixels are GC_ERR_UNSUPPORTED
 *     (2^36 u8 pixels are 64 GiB per image).
 *   - out may equal marker (in place, as the paper's filters run in place,
 *     Section 3.3).  out must not overlap mask (GC_ERR_ALIAS), and a partial
 *     overlap of out with marker is rejected too.
 *   - Work is enqueued on hip_stream (a hipStream_t; NULL = the null
 *     stream) and is asynchronous unless the entry point says otherwise.
 *   - The return value is GC_OK or a negative gc_status.  Arguments are
 *     validated before any HIP call; on error nothing is enqueued.
 *     gc_last_error() gives a detail message for the calling thread.
 *   - Calls that run concurrently on different streams are safe; each
 *     (device, stream) pair has its own workspace (gc_plan objects have
 *     their own), except gc_geodesic_chain_noalloc, whose calls on one
 *     device share one buffer.
 *   - The chain entry points (geodesic and plain) may be recorded into a
 *     HIP graph by stream capture once a call of at least the same size has
 *     run on the capturing stream (that call sizes the stream's workspace;
 *     a capture that would have to grow it returns GC_ERR_UNSUPPORTED).
 *     The graph keeps using the capturing stream's workspace: replays must
 *     not run at the same time as library calls on that stream (replaying
 *     on the capturing stream itself orders them).  A workspace that a
 *     capture has used is never freed: when a later call on that stream
 *     needs a larger one, the old buffer stays allocated until the process
 *     ends, so replays stay valid.  Entry points that read a convergence
 *     word on the host (reconstructions, the operators built on them, the
 *     quasi-distance transform) cannot be captured.
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
 * A batch of geodesic chains of equal shape (Eq. 3-4), all advanced by the
 * same launches: what gc_geodesic_{dilate,erode}_chain computes for each of
 * n_images images, image i at element offset i * image_stride from marker,
 * mask and out (image_stride >= (height - 1) * pitch + width when
 * n_images > 1; n_images <= 65535).  op = GC_DILATE or GC_ERODE.  out may
 * equal marker; out must not overlap mask, nor partially overlap marker.
 * ------------------------------------------------------------------- */
int gc_geodesic_chain_batch(gc_dtype dtype, gc_op op, const void *marker, const void *mask,
                            void *out, gc_shape shape, int32_t n_images, int64_t image_stride,
                            int64_t n_steps, void *hip_stream);

/* ---------------------------------------------------------------------
 * The geodesic chain for callers that cannot allocate device memory:
 * code recorded into a HIP graph by stream capture, serving loops that
 * must not allocate, harnesses that forbid hipMalloc.
 *
 * Computes what gc_geodesic_dilate_chain (op = GC_DILATE) or
 * gc_geodesic_erode_chain (op = GC_ERODE) computes, with the same
 * arguments, validation, aliasing rules and results, and calls no
 * hipMalloc, hipFree or other allocating routine.  Its ping-pong image
 * lives in a fixed array inside the library, one per device, held until
 * the process ends:
 *   - limit: the image's extent, ((height - 1) * pitch + width) elements,
 *     must fit 16 MiB (16777216 bytes: a 4096 x 4096 u8 image, 2048 x 2048
 *     f32, 1024 x 2048 f64); larger images return GC_ERR_UNSUPPORTED
 *     before any HIP call;
 *   - every call on one device shares that device's array: calls that
 *     overlap in time on one device (two streams, or a graph replay beside
 *     an eager call) race and give undefined results; the caller orders
 *     them.  The array needs no clearing between calls (each launch writes
 *     every pixel the next one reads);
 *   - the first call on a device looks the array's address up
 *     (hipGetSymbolAddress); make that first call outside stream capture.
 * The measurement hook (gc_profile_*) does not record these calls.
 * ------------------------------------------------------------------- */
int gc_geodesic_chain_noalloc(gc_dtype dtype, gc_op op, const void *marker,
                              const void *mask, void *out, gc_shape shape,
                              int64_t n_steps, void *hip_stream);

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
 * Reconstruction-based operators (Section 2, Eq. 6-12).
 *
 * Each runs ONE reconstruction with f as the mask, framed by pixelwise
 * passes; f is read-only and out receives the result (out must not overlap
 * f: GC_ERR_ALIAS).  Pixelwise arithmetic is done in the image's dtype:
 * u8 differences saturate at 0, f32/f64 differences are one IEEE
 * subtraction (h is first rounded to the dtype).  The border B of an image
 * is its first and last row and column.
 *
 * max_steps, *steps_out, GC_ERR_NOT_CONVERGED and the stream
 * synchronisation are those of the reconstruction calls above; when the cap
 * is reached the operator is formed from the capped chain and the status is
 * GC_ERR_NOT_CONVERGED.
 *
 *   gc_hmax   H-maxima (Eq. 6): reconstruction by dilation of f - h under f.
 *             h finite and >= 0; for u8 an integer (values above 255 act
 *             as 255).
 *   gc_dome   dome extraction (Eq. 7): f - HMAX_h(f).
 *   gc_hfill  hole filling (Eq. 8-9): reconstruction by erosion, above f, of
 *             the marker equal to f on B and to max f elsewhere.
 *   gc_raobj  removal of objects touching the border (Eq. 10-11): f minus
 *             the reconstruction by dilation, under f, of the marker equal
 *             to f on B and to min f elsewhere.
 *   gc_open_by_reconstruction  (Eq. 12): reconstruction by dilation, under
 *             f, of size plain 3x3 erosions of f (size >= 0).
 * ------------------------------------------------------------------- */
int gc_hmax(gc_dtype dtype, const void *f, void *out, gc_shape shape, double h,
            int64_t max_steps, int64_t *steps_out, void *hip_stream);
int gc_dome(gc_dtype dtype, const void *f, void *out, gc_shape shape, double h,
            int64_t max_steps, int64_t *steps_out, void *hip_stream);
int gc_hfill(gc_dtype dtype, const void *f, void *out, gc_shape shape,
             int64_t max_steps, int64_t *steps_out, void *hip_stream);
int gc_raobj(gc_dtype dtype, const void *f, void *out, gc_shape shape,
             int64_t max_steps, int64_t *steps_out, void *hip_stream);
int gc_open_by_reconstruction(gc_dtype dtype, const void *f, void *out, gc_shape shape,
                              int64_t size, int64_t max_steps, int64_t *steps_out,
                              void *hip_stream);

/* ---------------------------------------------------------------------
 * Granulometry and alternating sequential filters (Section 2, Eq. 16-20).
 *
 * gamma_s(f) = delta_s(eps_s(f)) is the opening of size s (s plain 3x3
 * erosions, then s plain 3x3 dilations), phi_s(f) = eps_s(delta_s(f)) the
 * closing.
 *
 * gc_granulometry: G[s] = sum over all pixels of gamma_s(f), for
 *   s = 0..s_max (gamma_0 = f), and PS[s] = G[s] - G[s+1] for
 *   s = 0..s_max-1 (the pattern spectrum).  G (s_max + 1 values) and PS
 *   (s_max values, may be NULL) are HOST arrays of double; the sums are
 *   accumulated in double in a fixed order (exact for u8 images), so repeated
 *   calls return identical values.  SYNCHRONISES hip_stream.
 * gc_asf: out = phi_smax(gamma_smax(... phi_1(gamma_1(f)))); s_max = 0
 *   copies f.  out may equal f; out must not partially overlap f.
 * ------------------------------------------------------------------- */
int gc_granulometry(gc_dtype dtype, const void *f, gc_shape shape, int32_t s_max,
                    double *G, double *PS, void *hip_stream);
int gc_asf(gc_dtype dtype, const void *f, void *out, gc_shape shape, int32_t s_max,
           void *hip_stream);

/* ---------------------------------------------------------------------
 * Quasi-distance transform (Section 2, Eq. 13-15; Algorithm 6).
 *
 * Applies plain 3x3 erosions eps_j = eps_1(eps_{j-1}(f)) until one changes
 * no pixel (at most max(X, Y) - 1 of them change anything).  For every
 * pixel, residual = the largest eps_{j-1}(f) - eps_j(f) over j (in f's
 * dtype) and d = the first j reaching it (0 where every residual is 0); a
 * later erosion replaces them only with a strictly larger residual.  With
 * lipschitz != 0, eta(g) = min(g, eps_1(g) + 1) is then applied to d until
 * it changes nothing (Eq. 14-15: where g exceeds its window minimum by more
 * than 1 it drops to that minimum + 1), giving the 1-Lipschitz d_L1.
 *
 *   f         input image (device, read-only).
 *   dist      int32 output, d_L1 (lipschitz != 0) or d (device, 4-byte
 *             aligned); element (x, y) at y * pitch + x, the same pitch in
 *             elements as f.
 *   residual  optional output of f's dtype, same pitch (NULL: not stored).
 *   *erosion_steps, *eta_steps (host, may be NULL): the erosions and eta
 *             applications that changed at least one pixel.
 *
 * dist and residual must not overlap f or each other (GC_ERR_ALIAS).  The
 * call SYNCHRONISES hip_stream (the chain lengths are data-dependent).
 * ------------------------------------------------------------------- */
int gc_quasi_distance(gc_dtype dtype, const void *f, int32_t *dist, void *residual,
                      gc_shape shape, int32_t lipschitz, int64_t *erosion_steps,
                      int64_t *eta_steps, void *hip_stream);

/* ---------------------------------------------------------------------
 * Batches: many independent chains (Eq. 4), each with its own image size
 * and number of steps, run by ONE persistent kernel launch recorded in a
 * HIP graph.  There is no batching in the paper; its closest analogue is
 * keeping many filters of a chain in flight at once (Section 3.5).
 *
 * gc_item: marker / mask / out are device pointers (same rules as the
 * single-image calls: out may equal marker, must not overlap mask).  All
 * items of one plan must be geodesic (mask != NULL) or all plain (mask ==
 * NULL).  n_steps >= 0 runs that many steps; n_steps < 0 (geodesic items
 * only) runs to stability, as gc_reconstruct_by_dilation / _erosion do for
 * one image (Eq. 5).
 *
 * gc_plan_create validates the items, chooses the tile family and steps per
 * block (from the autotuner's table when it has an entry for the items'
 * size class, see gc_autotune), builds the work list, allocates the plan's
 * workspace (two work images per item plus counters) and records the launch
 * into a HIP graph.  It copies the gc_item array; the images themselves
 * must stay allocated while the plan is used.  It synchronises the device
 * stream it uses for recording.  A plan whose work list (tiles x blocks
 * summed over the items) exceeds 2^31 - 1 is GC_ERR_UNSUPPORTED.
 *
 * gc_plan_launch replays the graph on hip_stream (asynchronous).  Launches
 * of one plan must not overlap each other (they share the workspace).
 * The kernel's workgroups draw work items in dependency order and wait
 * only for items drawn before theirs, so a launch finishes whatever part of
 * its grid is resident: plans may run at the same time on different
 * streams, or beside other work.  Every wait is also bounded (2 seconds);
 * past the bound the launch drains and gc_plan_status reports GC_ERR_HIP
 * (results invalid).
 * With run-to-stability items it is synchronous instead: each replay runs
 * every active image for 2 blocks of 20 steps while the kernel records, per
 * block, which steps changed a pixel; between replays the host retires the
 * images that reached a step without change (their result is then a fixed
 * point) and the others continue from their output.  Fixed-length items
 * finish in the first replay.  It returns GC_ERR_NOT_CONVERGED if an image
 * exceeds width x height + 1 steps, which a reconstruction cannot.
 *
 * gc_plan_steps writes, per item (host array of n_items), the steps of the
 * last launch: n_steps for fixed-length items, the number of steps that
 * changed a pixel for run-to-stability items (-1 before the first launch).
 *
 * gc_plan_status waits for the plan's last launch and returns GC_OK, or
 * GC_ERR_HIP if a dependency wait inside the kernel hit its safety bound
 * (results then invalid).
 *
 * gc_plan_info reports totals of the plan (any pointer may be NULL):
 * pixel-steps per launch of the fixed-length items, work items per replay,
 * workgroups launched, tile family and the largest steps-per-block used.
 *
 * gc_plan_tune times the kernel's launch shapes (tile family x steps per
 * block, the built-in choice among them) on scratch images with exactly
 * this plan's shapes and chain lengths -- the caller's images are not read
 * or written, so in-place items are safe -- and rebuilds the plan with the
 * fastest.  The handle stays valid; *best_ms (host, may be NULL) receives
 * the winner's time per launch.  Synchronises; allocates scratch for three
 * images per item while it runs.  Plans with run-to-stability items keep
 * the built-in shape (GC_ERR_UNSUPPORTED).
 * ------------------------------------------------------------------- */
typedef struct {
    const void *marker;
    const void *mask;
    void *out;
    gc_shape shape;
    int64_t n_steps;
} gc_item;

typedef struct gc_plan gc_plan;

int gc_plan_create(gc_dtype dtype, gc_op op, const gc_item *items, int32_t n_items,
                   gc_plan **plan_out);
int gc_plan_launch(gc_plan *plan, void *hip_stream);
int gc_plan_status(gc_plan *plan);
int gc_plan_steps(const gc_plan *plan, int64_t *steps);
int gc_plan_info(const gc_plan *plan, int64_t *px_steps, int64_t *work_items,
                 int32_t *workgroups, int32_t *tile, int32_t *block_steps);
int gc_plan_destroy(gc_plan *plan);
int gc_plan_tune(gc_plan *plan, double *best_ms);

/* ---------------------------------------------------------------------
 * Autotuner.  Times every candidate (tile family x steps per block) of the
 * persistent kernel on scratch images of the given size class and records
 * the fastest in a process-wide table that gc_plan_create consults (a plan
 * whose items all have entries takes the tile family with the least
 * predicted time and each item's steps per block for it; plans with
 * run-to-stability items and single-image chains keep their own launch
 * shapes).  Size class = (ceil(log2 width),
 * ceil(log2 height)).  geodesic != 0 tunes the geodesic kernel, else the
 * plain one.  Synchronises the device; allocates scratch memory.
 * best_tile / best_k (may be NULL) receive the choice.
 * ------------------------------------------------------------------- */
int gc_autotune(gc_dtype dtype, gc_op op, int32_t geodesic, int64_t width, int64_t height,
                int32_t *best_tile, int32_t *best_k);

/* Drop every autotuner entry. */
int gc_autotune_clear(void);

/* ---------------------------------------------------------------------
 * The autotuner's table as plain records, so that a later process can
 * reuse the timings instead of tuning again (the Python layer keeps them
 * in a JSON file: autotune_save / autotune_load).  One record per size
 * class: dtype, op, geodesic (0/1), the class (sides up to 2^log2_width x
 * 2^log2_height, log2 in 0..14), the chosen tile family, and per family
 * the steps per block and the measured rate in pixel-steps per second
 * (0 where a family was not timed).  Host memory, caller-owned; neither
 * call touches the GPU.
 *
 * gc_autotune_export copies at most cap records into out (out may be NULL
 * when cap is 0) and sets *count to the number the table holds.
 * gc_autotune_import adds the records, replacing those of the same class;
 * it checks them all first (known dtype, op and family; geodesic 0 or 1;
 * log2 sides in 0..14; steps per block in 0..63 with the chosen family's
 * at least 1; rates finite and >= 0) and on any bad record returns
 * GC_ERR_INVALID_ARG with the table unchanged.
 * ------------------------------------------------------------------- */
#define GC_TUNE_FAMILIES 5
typedef struct {
    int32_t dtype, op, geodesic;
    int32_t log2_width, log2_height;
    int32_t best_tile;
    int32_t k[GC_TUNE_FAMILIES];
    double rate[GC_TUNE_FAMILIES];
} gc_tune_entry;

int gc_autotune_export(gc_tune_entry *out, int32_t cap, int32_t *count);
int gc_autotune_import(const gc_tune_entry *entries, int32_t n);

/* ---------------------------------------------------------------------
 * Differentiation of a geodesic chain (not in the paper).  f32 and f64
 * only; values must be finite.
 *
 * Every output value of the chain is a copy of one input value (a marker
 * pixel or a mask pixel), so the chain is piecewise the identity on a
 * selection of its inputs.  gc_geodesic_chain_fwd_codes runs n_steps
 * geodesic steps like gc_geodesic_{dilate,erode}_chain and also writes, for
 * every step t and pixel p, a code naming where out_t(p) came from:
 *   (dy+1)*3 + (dx+1)  the FIRST extremal neighbour (dx, dy in -1..1) of
 *                      the clipped 3x3 window in raster (dy, dx) order;
 *   9                  the mask won the clamp (ties go to the mask).
 * codes: caller-owned device buffer of n_images * n_steps * height * width
 * bytes, dense, index ((i * n_steps + t) * height + y) * width + x.
 *
 * gc_geodesic_chain_bwd takes those codes and the gradient w.r.t. the
 * final state (grad_out) and WRITES grad_marker (gradient w.r.t. the state
 * before step 0) and ADDS the mask's gradient into grad_mask.  Each pixel
 * gathers the gradients of the neighbours whose codes point at it, visiting
 * them in raster order (the same order in which a raster-order scatter
 * would deliver them).  grad_marker must not overlap grad_out or grad_mask.
 * op names the chain the codes were recorded for (GC_DILATE or GC_ERODE,
 * else GC_ERR_INVALID_ARG); the codes already say which input each value
 * came from, so the arithmetic of the reverse pass is the same for both.
 *
 * Batches: n_images images of one shape, image i at element offset
 * i * image_stride from each image pointer (image_stride >= (height - 1) *
 * pitch + width when n_images > 1; n_images <= 65535).  Each launch (up to
 * 8 steps) covers the whole batch.  Images of more than 65535 * 112 rows
 * (f32) or 65535 * 80 rows (f64) return GC_ERR_UNSUPPORTED, for this call
 * and the source-id calls below.
 * ------------------------------------------------------------------- */
int gc_geodesic_chain_fwd_codes(gc_dtype dtype, gc_op op, const void *marker, const void *mask,
                                void *out, uint8_t *codes, gc_shape shape, int32_t n_images,
                                int64_t image_stride, int64_t n_steps, void *hip_stream);
int gc_geodesic_chain_bwd(gc_dtype dtype, gc_op op, const uint8_t *codes, const void *grad_out,
                          void *grad_marker, void *grad_mask, gc_shape shape, int32_t n_images,
                          int64_t image_stride, int64_t n_steps, void *hip_stream);

/* ---------------------------------------------------------------------
 * The same gradient through source ids (not in the paper): the per-step
 * routes above, composed over a run of steps.
 *
 * Following the codes of a pixel p of the final state backward through the
 * steps ends at a pixel of the state before step 0, or at the mask value of
 * some pixel (where the mask won a clamp): p's source, of which p's value
 * is a copy.  The gradient of sum(grad_out * out) w.r.t. marker pixel r is
 * the sum of grad_out(p) over the p whose source is marker pixel r, and
 * likewise for mask pixels; these are the sums gc_geodesic_chain_bwd forms
 * step by step, added in another order.
 *
 * gc_geodesic_chain_fwd_sources runs n_steps geodesic steps (out as in
 * gc_geodesic_{dilate,erode}_chain, n_steps = 0 copies) and writes, for
 * every pixel of out, its source id: the element offset y * pitch + x of the
 * source pixel within its image, with the top bit (0x80000000) set if the
 * source is the mask.  The choices are those of the codes (first extremal
 * neighbour in raster order, the mask winning ties).  sources:
 * caller-owned device buffer of uint32 with the images' layout (pitch and
 * image_stride in elements, as for the images).  Images may span at most
 * 2^31 - 1 elements each ((height - 1) * pitch + width), else
 * GC_ERR_UNSUPPORTED.  sources must not overlap the images.
 *
 * gc_geodesic_chain_bwd_sources WRITES grad_marker (zero, then every
 * pixel's grad_out added to the marker pixel its id names) and ADDS into
 * grad_mask (grad_out of the pixels whose source is a mask pixel, to that
 * pixel).  The additions into one pixel happen in an unspecified order
 * (hardware atomics), so results can differ between calls in the last
 * bits of the sums.  grad_marker, grad_mask, grad_out and sources must not
 * overlap.  An id whose offset lies beyond the image's elements
 * ((height - 1) * pitch + width) is ignored, so corrupted ids cannot make
 * the pass write outside the gradient images.  Batches as above (one
 * launch per 8 steps, and two launches for the reverse pass).
 * ------------------------------------------------------------------- */
int gc_geodesic_chain_fwd_sources(gc_dtype dtype, gc_op op, const void *marker, const void *mask,
                                  void *out, uint32_t *sources, gc_shape shape, int32_t n_images,
                                  int64_t image_stride, int64_t n_steps, void *hip_stream);
int gc_geodesic_chain_bwd_sources(gc_dtype dtype, const uint32_t *sources, const void *grad_out,
                                  void *grad_marker, void *grad_mask, gc_shape shape, int32_t n_images,
                                  int64_t image_stride, void *hip_stream);

/* ---------------------------------------------------------------------
 * Tuning hook: override the temporal-block depth (steps fused per launch)
 * and the tile family used by the chain kernels.  block_steps = 0 and
 * tile = -1 restore the built-in choice.  Process-wide; intended for the
 * autotuner and for tests that sweep launch shapes.
 * ------------------------------------------------------------------- */
int gc_set_tuning(int32_t block_steps, int32_t tile);

/* ---------------------------------------------------------------------
 * Large-window path for plain chains.  n plain 3x3 steps equal one
 * (2n+1) x (2n+1) window clipped to the image (Eq. 1-2, 4), computed
 * separably with the van Herk / Gil-Werman prefix-suffix scheme (the
 * size-insensitive method the introduction cites) at a cost per pixel that
 * does not depend on n; results are identical to the chain.  Plain chains
 * (gc_dilate_chain, gc_erode_chain and the plain chains inside the
 * composed operators) use it when n_steps >= min_steps and a line plus its
 * padding fits the kernel's 64 KiB LDS buffer.
 * min_steps: 0 = built-in crossover (26 steps for u8, 34 for f32, 38 for
 * f64), -1 = never, > 0 = that threshold.
 * Process-wide setting.
 * ------------------------------------------------------------------- */
int gc_set_window_path(int32_t min_steps);

/* ---------------------------------------------------------------------
 * Optional value check before a call.  The definitions (Section 2) are over
 * ordered values; NaN is not one, and the gradient entry points also need
 * finite values (the region's outside is held at -inf / +inf, which must
 * never tie with a pixel).  gc_validate_values scans a device image and
 * returns GC_ERR_INVALID_ARG if a pixel is a NaN, or an infinity when
 * allow_inf == 0 (gc_last_error says which); GC_OK otherwise, and always
 * for u8 and empty images.  Synchronises hip_stream (it reads one word
 * back).  The chain entry points do not call it themselves.
 * ------------------------------------------------------------------- */
int gc_validate_values(gc_dtype dtype, const void *image, gc_shape shape, int32_t allow_inf,
                       void *hip_stream);

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
