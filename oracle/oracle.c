/*
 * oracle.c -- plain, slow CPU oracle for chains of elementary 3x3 geodesic
 * dilations and erosions (Zlaus & Mongus, "Efficient method for parallel
 * computation of geodesic transformation on CPU", 2019).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; it exists so that tests and the benchmark's CPU baseline
 * can check the GPU library against the definitions of Section 2.
 *
 * Every function below is the textbook definition written out with naive
 * loops and two buffers (never in place):
 *
 *   - image domain P = {0..X-1} x {0..Y-1}, row-major, offset y*X + x
 *     (Section 2, first paragraph);
 *   - the 3x3 square structuring element w_1(p) is clipped to P, i.e. only
 *     neighbours inside the image take part (Section 2: w_s(p) is a subset
 *     of P);
 *   - erosion = min over the window, dilation = max over the reflected
 *     window (Eq. 1-2; the 3x3 square is symmetric, so reflection is a
 *     no-op);
 *   - elementary geodesic erosion  max(eps_1(f), m), dilation
 *     min(delta_1(f), m) (Eq. 3 and the sentence that defines its dual);
 *   - geodesic erosion/dilation of size s = s-fold composition (Eq. 4);
 *   - reconstruction = the limit of that composition (Eq. 5), detected as
 *     the first application that changes no pixel, which is the stopping
 *     rule of the convergence-detecting filter in Section 3.7 (Algorithm 5);
 *   - a reference gradient of the chain (not in the paper): every output
 *     value is a copy of exactly one input value, so the derivative routes
 *     each upstream gradient to the pixel (marker or mask) it was copied
 *     from.  Ties are broken by a fixed rule: the first extremal neighbour
 *     in raster (dy, dx) order, and the mask wins a tie with the
 *     neighbourhood extremum.  The gradient is formed by SCATTERING,
 *     deliberately different from the GPU's gather.
 *
 * All values are handled as double: u8, f32 and f64 inputs convert exactly
 * to double and min/max only select existing values, so every result
 * converts back exactly.  NaN inputs are outside the definition and are not
 * supported.
 *
 * Parity pins (tests/test_oracle_pins.py): brute-force clipped window
 * max/min, SE decomposition, threshold-decomposition flood fill for
 * reconstruction, invariants and dualities, special cases with known step
 * counts, exact finite differences and the value-identity gradient.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { ORACLE_DILATE = 0, ORACLE_ERODE = 1 };
enum { ORACLE_CODE_MASK = 9 };

void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* "a is better than b" for the operation: larger for dilation, smaller for
 * erosion. */
static int better(int op, double a, double b)
{
    return op == ORACLE_DILATE ? (a > b) : (a < b);
}

/* Extremum of f over the 3x3 window centred at (x, y), clipped to the image
 * (Eq. 1-2 with s = 1).  The window always contains its centre, so it is
 * never empty. */
static double window_extremum(int op, const double *f, int64_t X, int64_t Y,
                              int64_t x, int64_t y)
{
    double best = f[y * X + x];
    for (int64_t dy = -1; dy <= 1; ++dy) {
        int64_t yy = y + dy;
        if (yy < 0 || yy >= Y) continue;
        for (int64_t dx = -1; dx <= 1; ++dx) {
            int64_t xx = x + dx;
            if (xx < 0 || xx >= X) continue;
            double v = f[yy * X + xx];
            if (better(op, v, best)) best = v;
        }
    }
    return best;
}

/* The geodesic clamp of Eq. 3: dilation keeps min(delta_1(f), m), erosion
 * keeps max(eps_1(f), m).  A NULL mask means the plain (non-geodesic)
 * operator of Eq. 1-2. */
static double clamp_by_mask(int op, double v, const double *m, int64_t i)
{
    if (!m) return v;
    if (op == ORACLE_DILATE) return m[i] < v ? m[i] : v;
    return m[i] > v ? m[i] : v;
}

/* One elementary step: out = delta_1^m(f) or eps_1^m(f) (mask NULL: plain
 * delta_1 / eps_1).  Returns the number of pixels where out differs from f. */
int64_t oracle_step(int op, const double *f, const double *m, double *out,
                    int64_t X, int64_t Y)
{
    int64_t changed = 0;
#pragma omp parallel for reduction(+ : changed) schedule(static)
    for (int64_t y = 0; y < Y; ++y) {
        for (int64_t x = 0; x < X; ++x) {
            int64_t i = y * X + x;
            double v = clamp_by_mask(op, window_extremum(op, f, X, Y, x, y), m, i);
            out[i] = v;
            if (v != f[i]) ++changed;
        }
    }
    return changed;
}

/* Eq. 4: n-fold composition of the elementary step, two buffers.  n = 0
 * copies the marker unchanged. */
int oracle_chain(int op, const double *f, const double *m, double *out,
                 int64_t X, int64_t Y, int64_t n)
{
    size_t bytes = (size_t)X * (size_t)Y * sizeof(double);
    double *cur = (double *)malloc(bytes ? bytes : 1);
    double *nxt = (double *)malloc(bytes ? bytes : 1);
    if (!cur || !nxt) { free(cur); free(nxt); return -1; }
    memcpy(cur, f, bytes);
    for (int64_t t = 0; t < n; ++t) {
        oracle_step(op, cur, m, nxt, X, Y);
        double *tmp = cur; cur = nxt; nxt = tmp;
    }
    memcpy(out, cur, bytes);
    free(cur);
    free(nxt);
    return 0;
}

/* Eq. 5: apply the geodesic step until one application leaves every pixel
 * unchanged.  *steps_changed receives the number of applications that
 * changed at least one pixel, so out equals the chain of that length.
 * Returns 0 on convergence, 1 if max_steps applications all changed
 * something (out then holds the chain of length max_steps), -1 on
 * allocation failure.  max_steps < 0 means no limit. */
int oracle_reconstruct(int op, const double *f, const double *m, double *out,
                       int64_t X, int64_t Y, int64_t max_steps,
                       int64_t *steps_changed)
{
    size_t bytes = (size_t)X * (size_t)Y * sizeof(double);
    double *cur = (double *)malloc(bytes ? bytes : 1);
    double *nxt = (double *)malloc(bytes ? bytes : 1);
    if (!cur || !nxt) { free(cur); free(nxt); return -1; }
    memcpy(cur, f, bytes);
    int64_t count = 0;
    int status = 1;
    for (;;) {
        if (max_steps >= 0 && count >= max_steps) break;
        int64_t changed = oracle_step(op, cur, m, nxt, X, Y);
        if (changed == 0) { status = 0; break; }
        ++count;
        double *tmp = cur; cur = nxt; nxt = tmp;
    }
    if (status == 1 && X * Y > 0) {
        /* The cap was hit: one more look tells whether the last state is
         * already stable, in which case the reconstruction did converge. */
        if (oracle_step(op, cur, m, nxt, X, Y) == 0) status = 0;
    } else if (X * Y == 0) {
        status = 0;
    }
    memcpy(out, cur, bytes);
    *steps_changed = count;
    free(cur);
    free(nxt);
    return status;
}

/* Forward chain that also records, for every step t and pixel p, where the
 * output value came from: code (dy+1)*3 + (dx+1) of the FIRST extremal
 * neighbour in raster (dy, dx) order, or ORACLE_CODE_MASK when the mask
 * wins the clamp (ties go to the mask).  codes has n*Y*X entries, step-major.
 * out receives the final state. */
int oracle_chain_codes(int op, const double *f, const double *m, double *out,
                       uint8_t *codes, int64_t X, int64_t Y, int64_t n)
{
    size_t bytes = (size_t)X * (size_t)Y * sizeof(double);
    double *cur = (double *)malloc(bytes ? bytes : 1);
    double *nxt = (double *)malloc(bytes ? bytes : 1);
    if (!cur || !nxt) { free(cur); free(nxt); return -1; }
    memcpy(cur, f, bytes);
    for (int64_t t = 0; t < n; ++t) {
        uint8_t *ct = codes + (size_t)t * (size_t)X * (size_t)Y;
#pragma omp parallel for schedule(static)
        for (int64_t y = 0; y < Y; ++y) {
            for (int64_t x = 0; x < X; ++x) {
                int found = 0;
                double best = 0.0;
                int code = -1;
                for (int64_t dy = -1; dy <= 1; ++dy) {
                    int64_t yy = y + dy;
                    if (yy < 0 || yy >= Y) continue;
                    for (int64_t dx = -1; dx <= 1; ++dx) {
                        int64_t xx = x + dx;
                        if (xx < 0 || xx >= X) continue;
                        double v = cur[yy * X + xx];
                        if (!found || better(op, v, best)) {
                            best = v;
                            code = (int)((dy + 1) * 3 + (dx + 1));
                            found = 1;
                        }
                    }
                }
                int64_t i = y * X + x;
                if (m) {
                    int mask_wins = op == ORACLE_DILATE ? (m[i] <= best) : (m[i] >= best);
                    if (mask_wins) { best = m[i]; code = ORACLE_CODE_MASK; }
                }
                nxt[i] = best;
                ct[i] = (uint8_t)code;
            }
        }
        double *tmp = cur; cur = nxt; nxt = tmp;
    }
    memcpy(out, cur, bytes);
    free(cur);
    free(nxt);
    return 0;
}

/* Reverse pass of the chain by scattering: for t = n-1 .. 0, each pixel p
 * sends its gradient g_{t+1}(p) either to the mask (code 9, accumulated into
 * g_mask) or to the neighbour it copied from, which becomes part of g_t.
 * g_f receives g_0 (gradient w.r.t. the marker); g_mask is overwritten. */
int oracle_chain_grad(const uint8_t *codes, const double *g_out, double *g_f,
                      double *g_mask, int64_t X, int64_t Y, int64_t n)
{
    size_t npx = (size_t)X * (size_t)Y;
    size_t bytes = npx * sizeof(double);
    double *g = (double *)malloc(bytes ? bytes : 1);
    double *gp = (double *)malloc(bytes ? bytes : 1);
    if (!g || !gp) { free(g); free(gp); return -1; }
    memcpy(g, g_out, bytes);
    if (g_mask) memset(g_mask, 0, bytes);
    for (int64_t t = n - 1; t >= 0; --t) {
        const uint8_t *ct = codes + (size_t)t * npx;
        memset(gp, 0, bytes);
        /* Serial scatter: several pixels may send to the same source. */
        for (int64_t y = 0; y < Y; ++y) {
            for (int64_t x = 0; x < X; ++x) {
                int64_t i = y * X + x;
                int code = ct[i];
                if (code == ORACLE_CODE_MASK) {
                    if (g_mask) g_mask[i] += g[i];
                } else {
                    int64_t dy = code / 3 - 1, dx = code % 3 - 1;
                    gp[(y + dy) * X + (x + dx)] += g[i];
                }
            }
        }
        double *tmp = g; g = gp; gp = tmp;
    }
    memcpy(g_f, g, bytes);
    free(g);
    free(gp);
    return 0;
}
